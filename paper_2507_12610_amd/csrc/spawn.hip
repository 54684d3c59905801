// Particle spawning (Section 3.1 of the paper) for one simulation of a
// context: at the start of a step, up to N_spawn attempts while the count is
// below N_max.  Attempt a draws four 32-bit words of Philox4x32-10 (counter
// (a_lo, a_hi, 0, 0), key = the 64-bit seed): u = (k + 1/2) 2^-32 gives the
// centre s_min + u (s_max - s_min) per axis and the radius fraction of
// R_min + u (R_max - R_min); a radius carried over from a failed attempt is
// used instead of a new one.  A candidate fails if it would touch
// (R_j + r - d >= 0) a particle, including one placed earlier in the same
// step, or a mesh element of its simulation.
//
// Three kernels:
//   k_spawn_draw    the candidates of this step's attempts;
//   k_spawn_scan    every particle (and element) against every candidate: the
//                   smallest radius r for which the candidate would touch it,
//                   min-reduced per candidate.  The test R_j + r >= d after
//                   rounding is monotone in r, so "touches something already
//                   there" is exactly "r >= that minimum";
//   k_spawn_decide  one wave takes the attempts in order: the radius (new or
//                   carried), the threshold, then the particles accepted
//                   earlier in this step, and writes the new particles.
#include <hip/hip_runtime.h>

#include "sdem_internal.h"

namespace sdem {
namespace {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011).
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t a = c[0], b = c[2];
    const uint32_t ha = __umulhi(0xD2511F53u, a), la = 0xD2511F53u * a;
    const uint32_t hb = __umulhi(0xCD9E8D57u, b), lb = 0xCD9E8D57u * b;
    c[0] = hb ^ c[1] ^ k0;
    c[1] = lb;
    c[2] = ha ^ c[3] ^ k1;
    c[3] = la;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double unit_open(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// Smallest double r >= 0 with fl(Ra + r) >= d: bisection over the bit
// patterns of non-negative doubles (ordered like the values), 63 steps at
// most.  fl(Ra + d) >= d always holds, so d bounds it from above.
__device__ __forceinline__ double touch_radius(double Ra, double d) {
#pragma clang fp contract(off)
  if (Ra >= d) return 0.0;
  unsigned long long lo = 0ull, hi = (unsigned long long)__double_as_longlong(d);
  while (hi - lo > 1ull) {
    const unsigned long long mid = lo + ((hi - lo) >> 1);
    if (Ra + __longlong_as_double((long long)mid) >= d)
      hi = mid;
    else
      lo = mid;
  }
  return __longlong_as_double((long long)hi);
}

__global__ __launch_bounds__(kThreads) void k_spawn_draw(Ctx c) {
#pragma clang fp contract(off)
  const SpawnParams& P = *c.spawn;
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= P.n_spawn) return;
  const unsigned long long a = c.ctr->spawn_attempts + (unsigned long long)j;
  uint32_t w[4] = {(uint32_t)a, (uint32_t)(a >> 32), 0u, 0u};
  philox10(w, P.key[0], P.key[1]);
  double x[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = P.smin[k] + unit_open(w[k]) * (P.smax[k] - P.smin[k]);
  c.spawn_cand[j] = make_double4(x[0], x[1], x[2], unit_open(w[3]));
  c.spawn_thr[j] = 0x7FF0000000000000ull;  // +inf: nothing in the way yet
}

// Threads [0, n) take particle slots, threads [n, n + ntri) mesh elements.
__global__ __launch_bounds__(kThreads) void k_spawn_scan(Ctx c, State A) {
#pragma clang fp contract(off)
  const SpawnParams& P = *c.spawn;
  const int ns = P.n_spawn;
  __shared__ double4 cand[kSpawnMax];
  for (int j = threadIdx.x; j < ns; j += kThreads) cand[j] = c.spawn_cand[j];
  __syncthreads();
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t < c.n) {
    const double4 p = A.xr[t];
    // a particle farther than R + R_max from the spawn box reaches no
    // candidate (centres lie in the box up to rounding; generous margin)
    const double reach = (p.w + P.Rmax) * (1.0 + 1e-6);
    double e2 = 0.0;
    {
      const double px[3] = {p.x, p.y, p.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double e = fmax(fmax(P.smin[k] - px[k], px[k] - P.smax[k]), 0.0);
        e2 += e * e;
      }
    }
    if (e2 > reach * reach) return;
    const double lim = reach * reach;
    for (int j = 0; j < ns; ++j) {
      const double4 q = cand[j];
      const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 > lim) continue;  // no radius up to R_max touches
      const double r = touch_radius(p.w, sqrt(d2));
      atomicMin(&c.spawn_thr[j], (unsigned long long)__double_as_longlong(r));
    }
  } else if (t - c.n < c.ntri) {
    const int m = t - c.n;
    if (c.tri_sim[m] != P.sim) return;
    const double* tv = c.tri + 9 * m;
    const int nv = c.tri_nv[m];
    const double Rm = c.rmesh[m];
    for (int j = 0; j < ns; ++j) {
      const double4 q = cand[j];
      const double p3[3] = {q.x, q.y, q.z};
      double cp[3];
      closest_on_element(p3, tv, nv, cp);
      const double dx = q.x - cp[0], dy = q.y - cp[1], dz = q.z - cp[2];
      const double r = touch_radius(Rm, sqrt((dx * dx + dy * dy) + dz * dz));
      atomicMin(&c.spawn_thr[j], (unsigned long long)__double_as_longlong(r));
    }
  }
}

// One wave.  New particles go to slots n, n+1, ... with ids n, n+1, ...
// (one simulation per context when spawning, so slot count = id count).
__global__ __launch_bounds__(64) void k_spawn_decide(Ctx c, State A, Contacts cold) {
#pragma clang fp contract(off)
  const SpawnParams& P = *c.spawn;
  __shared__ double4 acc[kSpawnMax];
  const int lane = threadIdx.x;
  const int n0 = c.n;
  const double dR = P.Rmax - P.Rmin;
  double carried = c.ctr->spawn_carried;
  int made = 0, nacc = 0;
  for (int j = 0; j < P.n_spawn; ++j) {
    if ((int64_t)n0 + nacc >= P.n_max) break;
    ++made;
    const double4 q = c.spawn_cand[j];
    const double r = carried > 0.0 ? carried : P.Rmin + q.w * dR;
    bool blocked = r >= __longlong_as_double((long long)c.spawn_thr[j]);
    if (!blocked) {
      bool hit = false;
      for (int k = lane; k < nacc; k += 64) {
        const double4 b = acc[k];
        const double dx = b.x - q.x, dy = b.y - q.y, dz = b.z - q.z;
        const double d = sqrt((dx * dx + dy * dy) + dz * dz);
        hit = hit || (b.w + r) - d >= 0.0;
      }
      blocked = __any(hit);
    }
    // (blocked is the same in every lane)
    if (blocked) {
      carried = r;
    } else {
      carried = 0.0;
      if (lane == 0) acc[nacc] = make_double4(q.x, q.y, q.z, r);
      ++nacc;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int k = lane; k < nacc; k += 64) {
    const int slot = n0 + k;
    const double4 b = acc[k];
    Aux r;
    A.xr[slot] = b;
    A.q[slot] = make_double4(1.0, 0.0, 0.0, 0.0);
    r.vw[0] = make_double2(P.v0[0], P.v0[1]);
    r.vw[1] = make_double2(P.v0[2], P.w0[0]);
    r.vw[2] = make_double2(P.w0[1], P.w0[2]);
    r.pid = slot;
    r.prev = slot;
    r.off = 0;
    r.cnt = 0;
    A.a[slot] = r;
    cold.cnt[slot] = 0;
    cold.off[slot] = 0;
  }
  // slot groups that start to exist: no records, no statistics yet
  const int g0 = (n0 + kGroup - 1) / kGroup, g1 = (n0 + nacc + kGroup - 1) / kGroup;
  for (int g = g0 + lane; g < g1; g += 64) {
    c.gcnt[g] = 0;
    c.gstat[2 * g] = 0ull;
    c.gstat[2 * g + 1] = 0ull;
  }
  if (lane == 0) {
    c.ctr->spawn_attempts += (unsigned long long)made;
    c.ctr->spawn_carried = carried;
    c.ctr->spawn_new = nacc;
  }
}

// Radii by persistent id.
__global__ __launch_bounds__(kThreads) void k_scatter_radii(Ctx c, State S, double* R) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < c.n) {
    R[S.a[i].pid] = S.xr[i].w;
  }
}

inline int blocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_scatter_radii(const Ctx& c, const State& S, double* R, hipStream_t s) {
  if (c.n > 0) k_scatter_radii<<<blocks(c.n), kThreads, 0, s>>>(c, S, R);
  return hipGetLastError();
}

hipError_t launch_spawn(const Ctx& c, const State& A, const Contacts& cold, hipStream_t s) {
  hipError_t e = launch_mesh_now(c, s);
  if (e) return e;
  k_spawn_draw<<<blocks(kSpawnMax), kThreads, 0, s>>>(c);
  const int64_t work = (int64_t)c.n + c.ntri;
  if (work > 0) k_spawn_scan<<<blocks(work), kThreads, 0, s>>>(c, A);
  k_spawn_decide<<<1, 64, 0, s>>>(c, A, cold);
  return hipGetLastError();
}

}  // namespace sdem
