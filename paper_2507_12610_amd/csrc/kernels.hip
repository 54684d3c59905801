// HIP kernels of one DEM time step on gfx950 (MI355X).
//
// Step = bounding box -> grid -> cell keys + arrival ranks -> scan of the cell
// counts -> scatter -> stable reorder of the state into cell order -> narrow
// phase (one pass, wave-compacted contact records, partner lists) -> contact
// forces with spring carry-over (one lane per contact, no atomics) ->
// integration, which first gathers each particle's contact sums in a fixed
// order (so results do not depend on scheduling).
//
// Every kernel reads the context's flag word first and does nothing once a
// capacity or finiteness error has been raised, so a failed step leaves the
// previous step's buffers untouched.
#include <math.h>

#include <hip/hip_ext.h>

#include "sdem_internal.h"

namespace sdem {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_sum_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

__device__ __forceinline__ void raise_flag(Counters* ctr, int f) { atomicOr(&ctr->flags, f); }

// ---------------------------------------------------------------------------
// 1. bounding box of the centres, per simulation (Section 3.3)
// ---------------------------------------------------------------------------
// Per-wave segmented minimum of v[0..K) over runs of lanes with equal
// simulation; the first lane of each run gets the run's minima and the index
// of its partial: one partial per (wave, simulation) segment, in slot order.
// Must be called by every lane of a wave that holds at least one slot.
template <int K>
__device__ __forceinline__ bool wave_segment_min(const Ctx& c, int i, bool valid, double v[K],
                                                 int* bad, int* chunk) {
  const int lane = threadIdx.x & 63;
  const int sim = valid ? c.sim_of[i] : 0x7fffffff;
  if (!valid) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = INFINITY;
  }
  const int s0 = __shfl(sim, 0, 64);
  const int first = c.wchunk[i >> 6];
  if (__all(!valid || sim == s0)) {
    // the whole wave is one simulation: butterfly minimum
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int o = 32; o > 0; o >>= 1) v[k] = fmin(v[k], __shfl_xor(v[k], o, 64));
    *bad = __any(*bad) ? 1 : 0;
    *chunk = first;
    return lane == 0;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int os = __shfl_down(sim, o, 64);
    const int ob = __shfl_down(*bad, o, 64);
    const bool same = lane + o < 64 && os == sim;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double ov = __shfl_down(v[k], o, 64);
      if (same) v[k] = fmin(v[k], ov);
    }
    if (same) *bad |= ob;
  }
  const int prev = __shfl_up(sim, 1, 64);
  const bool head = valid && (lane == 0 || prev != sim);
  const unsigned long long heads = __ballot(head);
  *chunk = first + __popcll(heads & ((1ull << lane) - 1ull));
  return head;
}

// Bounding-box partials (Section 3.3: cells over the bounding box of the
// centres) of one wave; a non-finite coordinate turns the partial's minimum
// into NaN, which the grid kernel reports.
__device__ __forceinline__ void wave_bbox(const Ctx& c, int i, bool valid, double x, double y,
                                          double z) {
  double v[6] = {x, y, z, -x, -y, -z};  // minima of (x, y, z) and of (-x, -y, -z)
  int bad = valid && !(isfinite(x) && isfinite(y) && isfinite(z)) ? 1 : 0;
  int chunk;
  if (wave_segment_min<6>(c, i, valid, v, &bad, &chunk)) {
    double* p = c.part + kPart * (size_t)chunk;
    p[0] = bad ? NAN : v[0];
    p[1] = v[1];
    p[2] = v[2];
    p[3] = -v[3];
    p[4] = -v[4];
    p[5] = -v[5];
  }
}

// Largest drift from the binned centre over each (wave, simulation) segment.
__device__ __forceinline__ void wave_drift(const Ctx& c, int i, bool valid, double drift) {
  double v[1] = {-drift};
  int bad = 0, chunk;
  if (wave_segment_min<1>(c, i, valid, v, &bad, &chunk)) c.part[kPart * (size_t)chunk + 6] = -v[0];
}

__global__ __launch_bounds__(kThreads) void k_bbox_part(Ctx c, State A) {
  if (c.ctr->flags) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const bool valid = i < c.n;
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
  if (valid) p = A.xr[i];
  if (i - (int)(threadIdx.x & 63) < c.n) wave_bbox(c, i, valid, p.x, p.y, p.z);
}

// One workgroup of kGridThreads: one wave per simulation reduces that
// simulation's partials and lays out its grid (cells of edge h over the
// bounding box); then the grids are placed one after the other in the global
// cell table (exclusive scan of the cell counts over simulations).  Also
// opens the step: counts it and clears the contact allocation counter.
constexpr int kGridThreads = 1024;
constexpr int kMaxSims = 4096;

__device__ __forceinline__ void block_exclusive_scan_ll(long long* buf, int len, long long* total) {
  __shared__ long long tsum[kGridThreads];
  const int per = (len + kGridThreads - 1) / kGridThreads;
  const int b0 = threadIdx.x * per, b1 = min(len, b0 + per);
  long long s = 0;
  for (int i = b0; i < b1; ++i) s += buf[i];
  tsum[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kGridThreads; o <<= 1) {
    const long long y = threadIdx.x >= o ? tsum[threadIdx.x - o] : 0;
    __syncthreads();
    tsum[threadIdx.x] += y;
    __syncthreads();
  }
  long long run = tsum[threadIdx.x] - s;
  for (int i = b0; i < b1; ++i) {
    const long long v = buf[i];
    buf[i] = run;
    run += v;
  }
  if (threadIdx.x == kGridThreads - 1) *total = tsum[kGridThreads - 1];
  __syncthreads();
}

// Runs at the start of the steps that rebuild the cells (the first kernel
// after the bounding-box partials): counts the step as started.
__global__ __launch_bounds__(kGridThreads) void k_grid(Ctx c) {
  if (c.ctr->flags) return;
  __shared__ long long ncell[kMaxSims];
  __shared__ long long total;
  __shared__ int bad_total;
  if (threadIdx.x == 0) {
    bad_total = 0;
    atomicAdd(&c.ctr->steps, 1ull);  // steps started (the host discounts a failed one)
    c.ctr->rebuild_next = 0;
    c.ctr->rebuilds += 1ull;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = kGridThreads / 64;
  // grid of simulation s from the reduced bounding box (L, H)
  auto set_grid = [&](int s, const double* L, const double* H, bool bad) {
    SimGrid g;
    const double h = c.sp[s].h;
    long long nc = 1;
    for (int k = 0; k < 3; ++k) {
      g.lo[k] = 0.0;
      g.dim[k] = 1;
    }
    if (c.sp[s].np > 0) {
      for (int k = 0; k < 3; ++k) {
        const double ext = (H[k] - L[k]) / h;
        if (bad || !(ext >= 0.0) || !(ext < 1e30)) {
          bad = true;
        } else {
          const double dm = floor(ext) + 1.0;
          g.dim[k] = dm > 1048576.0 ? 1048576 : (int)dm;
          g.lo[k] = L[k];
        }
        nc *= (long long)g.dim[k];
      }
    }
    g.inv_h = 1.0 / h;
    g.cell_off = 0;
    c.sg[s] = g;
    ncell[s] = nc;
    if (bad) bad_total = 1;
  };
  if (c.nsims <= nw) {
    // few simulations: the whole workgroup reduces each one's partials
    __shared__ double red[kGridThreads / 64][6];
    __shared__ int redbad;
    for (int s = 0; s < c.nsims; ++s) {
      const int q0 = c.chunk0[s], q1 = c.chunk0[s + 1];
      double v[6] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
      bool bad = false;
      if (threadIdx.x == 0) redbad = 0;
      for (int q = q0 + (int)threadIdx.x; q < q1; q += kGridThreads) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double a = c.part[kPart * q + k];
          bad = bad || isnan(a);
          v[k] = fmin(v[k], a);
          v[3 + k] = fmin(v[3 + k], -c.part[kPart * q + 3 + k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 6; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] = fmin(v[k], __shfl_xor(v[k], o, 64));
      bad = __any(bad);
      __syncthreads();
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) red[wv][k] = v[k];
        if (bad) redbad = 1;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double L[3], H[3];
        for (int k = 0; k < 3; ++k) {
          double a = red[0][k], b = red[0][3 + k];
          for (int w = 1; w < nw; ++w) {
            a = fmin(a, red[w][k]);
            b = fmin(b, red[w][3 + k]);
          }
          L[k] = a;
          H[k] = -b;
        }
        set_grid(s, L, H, redbad != 0);
      }
    }
  } else {
    for (int s = wv; s < c.nsims; s += nw) {
      const int q0 = c.chunk0[s], q1 = c.chunk0[s + 1];
      double L[3] = {INFINITY, INFINITY, INFINITY}, H[3] = {-INFINITY, -INFINITY, -INFINITY};
      bool bad = false;
      for (int q = q0 + lane; q < q1; q += 64) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double a = c.part[kPart * q + k];
          bad = bad || isnan(a);
          L[k] = fmin(L[k], a);
          H[k] = fmax(H[k], c.part[kPart * q + 3 + k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k)
        for (int o = 32; o > 0; o >>= 1) {
          L[k] = fmin(L[k], __shfl_xor(L[k], o, 64));
          H[k] = fmax(H[k], __shfl_xor(H[k], o, 64));
        }
      bad = __any(bad);
      if (lane == 0) set_grid(s, L, H, bad);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < c.nchunks; q += kGridThreads) c.part[kPart * q + 6] = 0.0;
  block_exclusive_scan_ll(ncell, c.nsims, &total);
  for (int s = threadIdx.x; s < c.nsims; s += kGridThreads) {
    const long long off = ncell[s];
    c.sg[s].cell_off = (int)(off < 0x7fffffffLL ? off : 0x7fffffffLL);
  }
  if (threadIdx.x == 0) {
    const long long tot = total;
    c.ctr->ncells = (int)(tot < (long long)c.cap_cells ? tot : (long long)c.cap_cells);
    if (bad_total) raise_flag(c.ctr, kFlagNonFinite);
    if (tot > (long long)c.cap_cells) {
      c.ctr->need_cells = (int)(tot < 0x7fffffffLL ? tot : 0x7fffffffLL);
      raise_flag(c.ctr, kFlagCapCells);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. cell keys and arrival ranks (counting sort, pass 1)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(double x, double lo, double inv_h, int dim) {
  const double f = floor((x - lo) * inv_h);
  return f < 0.0 ? 0 : (f >= (double)dim ? dim - 1 : (int)f);
}

__global__ __launch_bounds__(kThreads) void k_keys(Ctx c, State A) {
  if (c.ctr->flags) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const SimGrid g = c.sg[c.sim_of[i]];
  const double4 p = A.xr[i];
  const int cx = cell_coord(p.x, g.lo[0], g.inv_h, g.dim[0]);
  const int cy = cell_coord(p.y, g.lo[1], g.inv_h, g.dim[1]);
  const int cz = cell_coord(p.z, g.lo[2], g.inv_h, g.dim[2]);
  const int key = g.cell_off + (cz * g.dim[1] + cy) * g.dim[0] + cx;
  c.key_tmp[i] = key;
  c.rank[i] = atomicAdd(&c.cell_cnt[key], 1);
  c.rowmax[key - cx] = 0ull;  // the reorder takes the maxima of occupied rows
}

// ---------------------------------------------------------------------------
// exclusive scan of the cell counts into cell starts, clearing the counts for
// the next step and writing the end entry.  Tables of up to kScanSmall cells:
// one workgroup; larger: block sums, a one-workgroup scan of them, downsweep.
// ---------------------------------------------------------------------------
constexpr int kScanSmall = 1 << 15;
constexpr int kScanOne = 1024;  // threads of the one-workgroup scan

__global__ __launch_bounds__(kScanOne) void k_scan_small(Ctx c) {
  if (c.ctr->flags) return;
  constexpr int kPer = 8;  // consecutive cells per thread and tile
  const int len = c.ctr->ncells;
  __shared__ int ws[kScanOne / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int base = 0; base < len; base += kScanOne * kPer) {
    const int i0 = base + threadIdx.x * kPer;
    int v[kPer];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      v[k] = i0 + k < len ? c.cell_cnt[i0 + k] : 0;
      sum += v[k];
    }
    const int x = wave_incl_scan(sum, lane);
    if (lane == 63) ws[wv] = x;
    __syncthreads();
    int run = carry + x - sum;
    for (int w = 0; w < wv; ++w) run += ws[w];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (i0 + k < len) {
        c.cell_start[i0 + k] = run;
        c.cell_cnt[i0 + k] = 0;
      }
      run += v[k];
    }
    __syncthreads();
    if (threadIdx.x == kScanOne - 1) carry = run;
    __syncthreads();
  }
  if (threadIdx.x == 0) c.cell_start[len] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Ctx c) {
  if (c.ctr->flags) return;
  const int len = c.ctr->ncells;
  const int chunk = (len + kScanBlocks - 1) / kScanBlocks;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(len, b0 + chunk);
  int s = 0;
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) s += c.cell_cnt[i];
  s = wave_sum_i32(s);
  __shared__ int ws[kScanThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += ws[w];
    c.scan_tmp[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(Ctx c) {
  if (c.ctr->flags) return;
  constexpr int per = kScanBlocks / kScanThreads;
  __shared__ int ws[kScanThreads / 64];
  int v[per];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = c.scan_tmp[threadIdx.x * per + k];
    sum += v[k];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int incl = wave_incl_scan(sum, lane);
  if (lane == 63) ws[wv] = incl;
  __syncthreads();
  int run = incl - sum;
  for (int w = 0; w < wv; ++w) run += ws[w];
#pragma unroll
  for (int k = 0; k < per; ++k) {
    c.scan_tmp[threadIdx.x * per + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) c.scan_tmp[kScanBlocks] = run;  // grand total
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(Ctx c) {
  if (c.ctr->flags) return;
  const int len = c.ctr->ncells;
  const int chunk = (len + kScanBlocks - 1) / kScanBlocks;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(len, b0 + chunk);
  __shared__ int ws[kScanThreads / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = c.scan_tmp[blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int base = b0; base < b1; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const int v = i < b1 ? c.cell_cnt[i] : 0;
    const int x = wave_incl_scan(v, lane);
    if (lane == 63) ws[wv] = x;
    __syncthreads();
    int pre = carry;
    for (int w = 0; w < wv; ++w) pre += ws[w];
    if (i < b1) {
      c.cell_start[i] = pre + x - v;
      c.cell_cnt[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {
      int t = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
      carry += t;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c.cell_start[len] = c.scan_tmp[kScanBlocks];
}

// ---------------------------------------------------------------------------
// 3. scatter (counting sort, pass 2) and stable reorder into cell order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_scatter(Ctx c) {
  if (c.ctr->flags) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  c.perm[c.cell_start[c.key_tmp[i]] + c.rank[i]] = i;
}

// Slot p of the scatter holds a particle of cell k; its final slot is the
// cell start plus the number of the cell's particles that came from a lower
// previous slot, so the order within a cell is the previous order (stable and
// deterministic).  Moves the whole state record.
__global__ __launch_bounds__(kThreads) void k_reorder(Ctx c, State A, State B, Contacts cold) {
  if (c.ctr->flags) return;
  // Thread d fills new slot d.  The scatter put the particles of each cell in
  // arrival order; slot d of cell k takes the particle whose previous slot
  // ranks d - cell_start[k] among them (stable order within a cell).
  const int d0 = blockIdx.x * kThreads;
  const int d = d0 + (int)threadIdx.x;
  __shared__ double2 st_x[kThreads * 2], st_v[kThreads * 3], st_q[kThreads * 2];
  int rk = -1 - (int)threadIdx.x;  // row of the slot's cell (unique dummy if none)
  double rr = 0.0;
  if (d < c.n) {
    const int k = c.key_tmp[c.perm[d]];
    const int cs = c.cell_start[k], ce = c.cell_start[k + 1];
    const int want = d - cs;
    int so = c.perm[d];
    for (int t = cs; t < ce; ++t) {
      const int v = c.perm[t];
      int r = 0;
      for (int u = cs; u < ce; ++u) r += (c.perm[u] < v) ? 1 : 0;
      if (r == want) {
        so = v;
        break;
      }
    }
    const double4 xr = A.xr[so], q = A.q[so];
    c.xb[d] = make_double4(xr.x, xr.y, xr.z, 0.0);  // binned centre
    const double2* vin = reinterpret_cast<const double2*>(A.vw + 6 * (size_t)so);
    const int t = threadIdx.x;
    st_x[2 * t] = make_double2(xr.x, xr.y);
    st_x[2 * t + 1] = make_double2(xr.z, xr.w);
    st_v[3 * t] = vin[0];
    st_v[3 * t + 1] = vin[1];
    st_v[3 * t + 2] = vin[2];
    st_q[2 * t] = make_double2(q.x, q.y);
    st_q[2 * t + 1] = make_double2(q.z, q.w);
    {
      const SimGrid g = c.sg[c.sim_of[d]];
      rk = k - (k - g.cell_off) % g.dim[0];
      rr = xr.w;
    }
    const int id = A.pid[so];
    B.pid[d] = id;
    c.key[d] = k;
    c.os[d] = make_int4(so, cold.off[so], cold.cnt[so], id);
  }
  // largest radius per cell row: slots are in row order, so a wave's rows
  // are runs of lanes; a segmented maximum leaves one atomic per run
  {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double ov = __shfl_down(rr, o, 64);
      const int ok = __shfl_down(rk, o, 64);
      if (lane + o < 64 && ok == rk) rr = fmax(rr, ov);
    }
    const int prev = __shfl_up(rk, 1, 64);
    if (rk >= 0 && (lane == 0 || prev != rk))
      atomicMax(&c.rowmax[rk], (unsigned long long)__double_as_longlong(rr));
  }
  __syncthreads();
  const int np = min(c.n - d0, kThreads);
  double2* gx = reinterpret_cast<double2*>(B.xr + d0);
  double2* gv = reinterpret_cast<double2*>(B.vw + 6 * (size_t)d0);
  double2* gq = reinterpret_cast<double2*>(B.q + d0);
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gx[k] = st_x[k];
  for (int k = threadIdx.x; k < 3 * np; k += kThreads) gv[k] = st_v[k];
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gq[k] = st_q[k];
}

// ---------------------------------------------------------------------------
// 4. mesh: the motion of each element's group (rotation about a centre and
//    harmonic displacement: an extension for rotating drums and vibrated
//    bases), the wall record read by the contact law, and plane data (the
//    plane through the stored slots 0, 1, 2: a triangle's, or a rectangle's
//    through corners 0, 1 and 3)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mesh(Ctx c, int all, int started) {
#pragma clang fp contract(off)
  if (c.ctr->flags) return;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= c.ntri) return;
  const SimParams& P = c.sp[c.tri_sim[m]];
  const MeshMotion& G = c.motion[c.tri_grp[m]];
  double* t = c.tri + 9 * m;
  const double* t0 = c.tri_ref + 9 * m;
  double* mv = c.tri_mv + 9 * m;
  if (all) {  // set-up: vertices at t = 0, no wall motion recorded yet
    for (int k = 0; k < 9; ++k) {
      t[k] = t0[k];
      mv[k] = 0.0;
    }
  } else if (G.moving) {
    // rigid motion at the time of the start of this step (`started`: the
    // step counter already counts it): turn by |omega| t about the axis
    // through the displaced centre, displacement d(t) with velocity d'(t)
    const double tm = (double)(c.ctr->steps - (unsigned long long)started) * P.dt;
    const double wv = 2.0 * kPi * G.freq;
    const double ph = wv * tm + G.phase;
    const double s1 = sin(ph) - sin(G.phase), c1 = wv * cos(ph);
    const double d[3] = {G.amp[0] * s1, G.amp[1] * s1, G.amp[2] * s1};
    const double wl = sqrt((G.omega[0] * G.omega[0] + G.omega[1] * G.omega[1]) +
                           G.omega[2] * G.omega[2]);
    if (wl > 0.0) {
      const double kx = G.omega[0] / wl, ky = G.omega[1] / wl, kz = G.omega[2] / wl;
      const double ang = wl * tm;
      const double co = cos(ang), si = sin(ang);
      for (int v = 0; v < 3; ++v) {
        const double rx = t0[3 * v] - G.center[0], ry = t0[3 * v + 1] - G.center[1],
                     rz = t0[3 * v + 2] - G.center[2];
        const double cx = ky * rz - kz * ry, cy = kz * rx - kx * rz, cz = kx * ry - ky * rx;
        const double kd = (kx * rx + ky * ry) + kz * rz;
        t[3 * v] = (G.center[0] + d[0]) + ((rx * co + cx * si) + kx * kd * (1.0 - co));
        t[3 * v + 1] = (G.center[1] + d[1]) + ((ry * co + cy * si) + ky * kd * (1.0 - co));
        t[3 * v + 2] = (G.center[2] + d[2]) + ((rz * co + cz * si) + kz * kd * (1.0 - co));
      }
    } else {
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) t[3 * v + k] = t0[3 * v + k] + d[k];
    }
    for (int k = 0; k < 3; ++k) {
      mv[k] = G.omega[k];
      mv[3 + k] = G.center[k] + d[k];
      mv[6 + k] = G.amp[k] * c1;
    }
  } else {
    return;
  }
  const double e1x = t[3] - t[0], e1y = t[4] - t[1], e1z = t[5] - t[2];
  const double e2x = t[6] - t[0], e2y = t[7] - t[1], e2z = t[8] - t[2];
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double nl = sqrt(nx * nx + ny * ny + nz * nz);
  if (nl > 0.0) {
    nx /= nl;
    ny /= nl;
    nz /= nl;
    c.tri_pl[4 * m] = nx;
    c.tri_pl[4 * m + 1] = ny;
    c.tri_pl[4 * m + 2] = nz;
    c.tri_pl[4 * m + 3] = nx * t[0] + ny * t[1] + nz * t[2];
  } else {  // point, segment or degenerate element: no plane filter
    c.tri_pl[4 * m] = 0.0;
    c.tri_pl[4 * m + 1] = 0.0;
    c.tri_pl[4 * m + 2] = 0.0;
    c.tri_pl[4 * m + 3] = 0.0;
  }
}

// Element bins (the mesh side of the broad phase): count, scan, fill and
// sort the (bin, element) pairs.  An element enters every bin of its grid
// that its vertex bounding box, grown by R_max + half skin + R_m of its
// simulation, overlaps; the margin on the growth covers rounding of the box
// ends, so a particle centre within R_i + R_m of the element lies in one of
// them, and so does a centre within R_i + R_m + half skin (the reach at
// which a rebuild records elements in the candidate lists).
__device__ __forceinline__ void tri_bins(const Ctx& c, int m, const MeshGrid& G, int i0[3],
                                         int i1[3]) {
  const double* t = c.tri + 9 * m;
  const bool rect = c.tri_nv[m] == 4;
  const SimParams& P = c.sp[c.tri_sim[m]];
  const double reach = ((P.rmax + P.half_skin) + c.rmesh[m]) * (1.0 + 1e-9);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = t[k], b = t[3 + k], e = t[6 + k];
    double mn = fmin(a, fmin(b, e)), mx = fmax(a, fmax(b, e));
    if (rect) {  // the implied fourth corner of a rectangle
      const double f = (b + e) - a;
      mn = fmin(mn, f);
      mx = fmax(mx, f);
    }
    const double pad = reach + 1e-12 * (fabs(mn) + fabs(mx));
    const double f0 = ((mn - pad) - G.lo[k]) * G.inv_h;
    const double f1 = ((mx + pad) - G.lo[k]) * G.inv_h;
    const int d = G.dim[k];
    i0[k] = f0 <= 0.0 ? 0 : (f0 >= (double)d ? d - 1 : (int)f0);
    i1[k] = f1 <= 0.0 ? 0 : (f1 >= (double)d ? d - 1 : (int)f1);
  }
}

__global__ __launch_bounds__(kThreads) void k_bin_count(Ctx c) {
  if (c.ctr->flags) return;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= c.ntri) return;
  const MeshGrid G = c.mg[c.tri_sim[m]];
  int i0[3], i1[3];
  tri_bins(c, m, G, i0, i1);
  for (int z = i0[2]; z <= i1[2]; ++z)
    for (int y = i0[1]; y <= i1[1]; ++y)
      for (int x = i0[0]; x <= i1[0]; ++x)
        atomicAdd(&c.bin_cnt[G.off + (z * G.dim[1] + y) * G.dim[0] + x], 1);
}

// Exclusive scan of the bin counts by one workgroup (a contiguous run of
// bins per thread); clears the counts for the fill.
__global__ __launch_bounds__(kBinScanThreads) void k_bin_scan(Ctx c) {
  if (c.ctr->flags) return;
  __shared__ int wsum[kBinScanThreads / 64];
  const int nb = c.nbins;
  const int per = (nb + kBinScanThreads - 1) / kBinScanThreads;
  const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += c.bin_cnt[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int incl = wave_incl_scan(sum, lane);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    int v = lane < kBinScanThreads / 64 ? wsum[lane] : 0;
    v = wave_incl_scan(v, lane);
    if (lane < kBinScanThreads / 64) wsum[lane] = v;
  }
  __syncthreads();
  int run = (incl - sum) + (w > 0 ? wsum[w - 1] : 0);
  for (int b = b0; b < b1; ++b) {
    const int k = c.bin_cnt[b];
    c.bin_start[b] = run;
    c.bin_cnt[b] = 0;
    run += k;
  }
  if (threadIdx.x == kBinScanThreads - 1) {
    c.bin_start[nb] = run;
    if (run > c.cap_bin_entries) raise_flag(c.ctr, kFlagCapBins);
  }
}

__global__ __launch_bounds__(kThreads) void k_bin_fill(Ctx c) {
  if (c.ctr->flags) return;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= c.ntri) return;
  const MeshGrid G = c.mg[c.tri_sim[m]];
  int i0[3], i1[3];
  tri_bins(c, m, G, i0, i1);
  for (int z = i0[2]; z <= i1[2]; ++z)
    for (int y = i0[1]; y <= i1[1]; ++y)
      for (int x = i0[0]; x <= i1[0]; ++x) {
        const int b = G.off + (z * G.dim[1] + y) * G.dim[0] + x;
        const int pos = c.bin_start[b] + atomicAdd(&c.bin_cnt[b], 1);
        if (pos < c.cap_bin_entries) c.bin_tri[pos] = m;
      }
}

// Ascending triangle order within each bin (the fill order is arbitrary), so
// that the narrow phase visits triangles in the same order every run.
__global__ __launch_bounds__(kThreads) void k_bin_sort(Ctx c) {
  if (c.ctr->flags) return;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= c.nbins) return;
  const int s0 = c.bin_start[b], s1 = c.bin_start[b + 1];
  for (int i = s0 + 1; i < s1; ++i) {
    const int v = c.bin_tri[i];
    int j = i - 1;
    while (j >= s0 && c.bin_tri[j] > v) {
      c.bin_tri[j + 1] = c.bin_tri[j];
      --j;
    }
    c.bin_tri[j + 1] = v;
  }
  c.bin_cnt[b] = 0;
}

// ---------------------------------------------------------------------------
// 5. narrow phase (Section 3.3), one pass.  SUB adjacent lanes share one
//    particle slot s and split its search (every SUB-th triangle of its bin
//    and every SUB-th cell row of its search box), which shortens each
//    lane's chain of dependent loads in the latency-bound search.  Partners
//    are the particles with a higher slot in the cells within R_s + R_max of
//    x_s on each axis: with cells in (z, y, x) row order each row of that box
//    is one contiguous slot range, and rows before the own row hold only
//    lower slots.  Each pair is thus found once, by its lower slot (the
//    owner).  Hits go to a per-lane list in LDS; a wave prefix scan gives
//    every lane its place (a slot's SUB lists end up adjacent) and one atomic
//    per wave reserves the wave's records.  Pair records are also entered in
//    the partner's list (one integer atomic per pair).
// ---------------------------------------------------------------------------
// The search of logical block blk.  LDS comes from the caller: the hit lists,
// the drift reach per simulation, a reduction buffer and the wave totals.
// With FUSED (one lane per slot), the group's first kThreads records are also
// left in LDS (rec_a: owner slot within the group, rec_b: partner).  Returns
// the group's record count (one lane per slot; 0 otherwise), or -1 when an
// earlier failure is flagged.
template <int SUB, bool FUSED>
__device__ __forceinline__ int detect_group(const Ctx& c, const State& A, const State& B,
                                            const Contacts& cn, const int rebuilt, const int blk,
                                            int (*hits)[kMaxOwn][64], double* xdrift, double* red,
                                            int* wtots, unsigned char* rec_a, int* rec_b) {
  // the sorted copy when this step rebuilt the cells, else the kept order
  const State S = rebuilt ? B : A;
  const int n = c.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bg = blk * kThreads;
  const int g = bg + threadIdx.x;
  const int s = g / SUB, sub = g % SUB;
  // The own centre, simulation and candidate list head are loaded before the
  // failure flag is examined (a step after a failed one exits there): none
  // depends on the step's outcome so far.  List entries are only followed
  // within the recorded count.
  int sim = 0, vcnt0 = -1, vraw[4] = {s, s, s, s};
  double4 ps = make_double4(0.0, 0.0, 0.0, 0.0);
  if (s < n) {
    sim = c.nsims == 1 ? 0 : c.sim_of[s];
    ps = S.xr[s];
    if (c.skin_on && !rebuilt) {
      vcnt0 = c.vcnt[g];
#pragma unroll
      for (int u = 0; u < 4; ++u) vraw[u] = c.vlist[(size_t)u * c.vstride + g];
    }
  }
  // A wave that sees a failure flagged searches nothing.  Another workgroup
  // may raise a flag while this one starts, so with one lane per slot a
  // wave that sees it still posts a zero total for the workgroup's record
  // offsets before it leaves: the records of the waves that go on stay
  // consistent (the step is failed and repeated anyway).
  const bool dead = c.ctr->flags != 0;
  if (dead && SUB != 1) return -1;
  // a step that keeps the cells starts here (and is counted if its searches
  // must reach past the skin)
  if (!rebuilt && !dead && blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd(&c.ctr->steps, 1ull);
    if (c.ctr->rebuild_next) c.ctr->drift_steps += 1ull;
  }
  // If a particle drifted past half the skin since the cells were built,
  // every search of this step reaches by the excess further: the largest
  // drift of each simulation of this workgroup, from the integration's
  // per-wave partials (a rare step; the others skip this).
  int sim_lo = 0;
  if (!rebuilt && c.ctr->rebuild_next && bg / SUB < n) {
    sim_lo = c.sim_of[bg / SUB];
    const int sim_hi = c.sim_of[min(n - 1, (bg + kThreads - 1) / SUB)];
    for (int sm = sim_lo; sm <= sim_hi; ++sm) {
      double dmax = 0.0;
      for (int q = c.chunk0[sm] + threadIdx.x; q < c.chunk0[sm + 1]; q += kThreads)
        dmax = fmax(dmax, c.part[kPart * q + 6]);
      for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
      __syncthreads();
      if (lane == 0) red[wv] = dmax;
      __syncthreads();
      if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, red[w]);
        const double ex = m - c.sp[sm].half_skin;
        xdrift[sm - sim_lo] = ex > 0.0 ? ex * (1.0 + 1e-6) : 0.0;
      }
    }
    __syncthreads();
  }
  int npp = 0, npw = 0;
  if (s < n && !dead) {
    const SimGrid gr = c.sg[sim];
    const double extra = (!rebuilt && c.ctr->rebuild_next) ? xdrift[sim - sim_lo] : 0.0;
    const double xs = ps.x, ys = ps.y, zs = ps.z, Rs = ps.w;
    // Between rebuilds, with no drift past half the skin in this simulation,
    // the candidates recorded at the last rebuild suffice: every particle
    // within R_s + R_t + 2 (half skin) of x_s then, and (static meshes) every
    // triangle within R_s + R_m + half skin.
    const double hsk = c.sp[sim].half_skin;
    const bool listed = c.skin_on && !rebuilt && extra == 0.0;
    const bool record = c.skin_on && rebuilt;
    const bool tri_listed = !c.sp[sim].moving;
    // entry k of this lane's candidate list
    auto vl = [&](int k) -> int& { return c.vlist[(size_t)k * c.vstride + g]; };
    const int nlist = listed ? vcnt0 : -1;
    int ncand = 0;
    auto test_wall = [&](int m) {
      const double p[3] = {xs, ys, zs};
      double cp[3];
      closest_on_element(p, c.tri + 9 * m, c.tri_nv[m], cp);
      double dx, dy, dz, d;
      const double delta = pair_gap(xs, ys, zs, Rs, cp[0], cp[1], cp[2], c.rmesh[m], &dx, &dy, &dz, &d);
      if (delta >= 0.0) {
        if (npw + npp < kMaxOwn) hits[wv][npw + npp][lane] = -1 - m;
        ++npw;
      }
      return d;
    };
    auto test = [&](int t, const double4& pt) {
      const double ex = xs - pt.x, ey = ys - pt.y, ez = zs - pt.z;
      const double sr = Rs + pt.w;
      // cheap conservative reject before the exactly rounded test
      if ((ex * ex + ey * ey) + ez * ez > sr * sr * (1.0 + 1e-9)) return;
      double dx, dy, dz, d;
      const double delta = pair_gap(xs, ys, zs, Rs, pt.x, pt.y, pt.z, pt.w, &dx, &dy, &dz, &d);
      if (delta >= 0.0) {
        if (npw + npp < kMaxOwn) hits[wv][npw + npp][lane] = t;
        ++npp;
      }
    };
    // ---- triangles listed in the bin of x_s (unless the list holds them)
    if (!(nlist >= 0 && tri_listed)) {
      int k0 = 0, k1 = 0;
      if (c.sp[sim].ntri > 0) {
        const MeshGrid G = c.mg[sim];
        const double fx = (xs - G.lo[0]) * G.inv_h, fy = (ys - G.lo[1]) * G.inv_h,
                     fz = (zs - G.lo[2]) * G.inv_h;
        if (fx >= 0.0 && fy >= 0.0 && fz >= 0.0 && fx < (double)G.dim[0] &&
            fy < (double)G.dim[1] && fz < (double)G.dim[2]) {
          const int b = G.off + ((int)fz * G.dim[1] + (int)fy) * G.dim[0] + (int)fx;
          k0 = c.bin_start[b];
          k1 = c.bin_start[b + 1];
        }
      }
      const bool rec_tri = record && tri_listed;
      for (int k = k0 + sub; k < k1; k += SUB) {
        const int m = c.bin_tri[k];
        const double* pl = c.tri_pl + 4 * m;
        const double reach = (Rs + c.rmesh[m]) + (rec_tri ? hsk : 0.0);
        const double pd = (pl[0] * xs + pl[1] * ys + pl[2] * zs) - pl[3];
        if (fabs(pd) > reach * (1.0 + 1e-9) + 1e-300) continue;
        const double d = test_wall(m);
        if (rec_tri && d <= reach * (1.0 + 1e-9)) {
          if (ncand < kCand) vl(ncand) = -1 - m;
          ++ncand;
        }
      }
    }
    // ---- particles (and listed triangles)
    if (nlist >= 0) {
      // four candidates per iteration; the next four slots are loaded while
      // these are tested (slots past the list read the own slot)
      int tn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) tn[u] = u < nlist ? vraw[u] : s;
      for (int k = 0; k < nlist; k += 4) {
        int tt[4];
        double4 pt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) tt[u] = tn[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) pt[u] = S.xr[tt[u] >= 0 ? tt[u] : s];
#pragma unroll
        for (int u = 0; u < 4; ++u) tn[u] = k + 4 + u < nlist ? vl(k + 4 + u) : s;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (k + u >= nlist) continue;
          if (tt[u] >= 0)
            test(tt[u], pt[u]);
          else
            (void)test_wall(-1 - tt[u]);
        }
      }
    } else {
    // The half-shell rows run from the own row through the
    // rest of the own (y, z) plane, then over the full planes above; lane
    // `sub` takes every SUB-th of them.  A row is searched over the x cells
    // within rho = R_s + (largest radius in the row) of x_s, given its (y, z)
    // distance from x_s; rows farther than rho are skipped.  The row geometry
    // is done in cell units relative to the own cell, in float, with margins
    // (1e-5 cell, 1e-6 relative) far above its rounding, so the search only
    // ever widens.  The largest radius of a row is loaded two rows ahead and
    // the slot range one row ahead of the candidates being examined.
    const int loc = c.key[s] - gr.cell_off;
    const int nx = gr.dim[0], ny = gr.dim[1], nz = gr.dim[2];
    const int cx = loc % nx, cyz = loc / nx, cy = cyz % ny, cz = cyz / ny;
    const float fx = (float)((xs - gr.lo[0]) * gr.inv_h - cx);
    const float fy = (float)((ys - gr.lo[1]) * gr.inv_h - cy);
    const float fz = (float)((zs - gr.lo[2]) * gr.inv_h - cz);
    // drift allowed since the cells were built (plus any excess measured);
    // a rebuild step looks twice as far to record the candidates
    const double hs = record ? 2.0 * hsk : hsk + extra;
    const double reach = ((Rs + c.sp[sim].rmax) + hs) * (1.0 + 1e-9);
    const int y0 = cell_coord(ys - reach, gr.lo[1], gr.inv_h, ny);
    const int y1 = cell_coord(ys + reach, gr.lo[1], gr.inv_h, ny);
    const int z1 = cell_coord(zs + reach, gr.lo[2], gr.inv_h, nz);
    auto step1 = [&](int* zz, int* yy) {
      if (++*yy > y1) {
        ++*zz;
        *yy = y0;
      }
    };
    auto advance = [&](int* zz, int* yy) {
#pragma unroll
      for (int k = 0; k < SUB; ++k) step1(zz, yy);
    };
    auto row_at = [&](int zz, int yy) { return gr.cell_off + (zz * ny + yy) * nx; };
    auto load_rm = [&](int zz, int yy) {
      return zz <= z1 ? __longlong_as_double((long long)c.rowmax[row_at(zz, yy)]) : 0.0;
    };
    auto bounds = [&](int zz, int yy, double rm, int* t0, int* t1) {
      *t0 = 0;
      *t1 = 0;
      if (zz > z1) return;
      const float ry = (float)(yy - cy), rz = (float)(zz - cz);
      const float dy = fmaxf(fmaxf(ry - fy, fy - (ry + 1.0f)) - 1e-5f, 0.0f);
      const float dz = fmaxf(fmaxf(rz - fz, fz - (rz + 1.0f)) - 1e-5f, 0.0f);
      const float rho = (float)(((Rs + rm) + hs) * gr.inv_h) * (1.0f + 1e-6f) + 1e-5f;
      const float d2 = dy * dy + dz * dz;
      if (d2 > rho * rho) return;
      const float xr = sqrtf(rho * rho - d2) * (1.0f + 1e-6f) + 1e-5f;
      const int x0 = max(0, cx + (int)floorf(fx - xr));
      const int x1 = min(nx - 1, cx + (int)floorf(fx + xr));
      if (x1 < x0) return;
      const int row = row_at(zz, yy);
      *t0 = (zz == cz && yy == cy) ? s + 1 : c.cell_start[row + x0];
      *t1 = c.cell_start[row + x1 + 1];
    };
    // rows: C (candidates now), B (slot range next), A (largest radius next)
    int zA = cz, yA = cy;
    for (int k = 0; k < sub; ++k) step1(&zA, &yA);
    int zB = zA, yB = yA;
    double rmB = load_rm(zB, yB);
    advance(&zA, &yA);
    double rmA = load_rm(zA, yA);
    int t0n, t1n;
    bounds(zB, yB, rmB, &t0n, &t1n);
    int zC = zB;
    zB = zA;
    yB = yA;
    rmB = rmA;
    advance(&zA, &yA);
    rmA = load_rm(zA, yA);
    while (zC <= z1) {
      const int t0 = t0n, t1 = t1n;
      bounds(zB, yB, rmB, &t0n, &t1n);
      zC = zB;
      zB = zA;
      yB = yA;
      rmB = rmA;
      advance(&zA, &yA);
      rmA = load_rm(zA, yA);
      // four candidates per iteration so that four loads are in flight
      for (int t = t0; t < t1; t += 4) {
        double4 pt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pt[u] = S.xr[t + u < t1 ? t + u : t];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (t + u >= t1) break;
          if (record) {
            const double ex = xs - pt[u].x, ey = ys - pt[u].y, ez = zs - pt[u].z;
            const double sr = (Rs + pt[u].w) + 2.0 * hsk;
            if ((ex * ex + ey * ey) + ez * ez <= sr * sr * (1.0 + 1e-9)) {
              if (ncand < kCand) vl(ncand) = t + u;
              ++ncand;
            }
          }
          test(t + u, pt[u]);
        }
      }
    }
    if (record) c.vcnt[g] = ncand <= kCand ? ncand : -1;  // -1: search the cells
    }
  }
  // wave compaction: prefix scan of the per-lane counts, then one atomic per
  // wave on the counter of the wave's slot group (a wave's slots lie in one
  // group, and a group's counter sees at most 4*SUB waves)
  const int total_hits = npw + npp;
  const int mine = total_hits < kMaxOwn ? total_hits : kMaxOwn;
  const int incl = wave_incl_scan(mine, lane);
  const int wtot = __shfl(incl, 63, 64);
  const int grp = __shfl(g / SUB, 0, 64) >> kGroupShift;
  int base = 0, tot = 0;
  if (SUB == 1) {
    // one lane per slot: the workgroup is the slot group, so the waves'
    // offsets come from a scan of their totals, in slot order
    if (lane == 63) wtots[wv] = wtot;
    __syncthreads();
    for (int w = 0; w < kThreads / 64; ++w) {
      if (w < wv) base += wtots[w];
      tot += wtots[w];
    }
    if (threadIdx.x == 0 && grp < c.ngroups && !dead) c.gcnt[grp] = tot;
    if (dead) return -1;
  } else {
    if (lane == 63 && wtot > 0 && grp < c.ngroups) base = atomicAdd(&c.gcnt[grp], wtot);
    base = __shfl(base, 63, 64);
  }
  const int first = grp * c.gcap + base + incl - mine;
  // end of this slot's records: the last of its SUB lanes
  const int slot_end = __shfl(first + mine, (lane | (SUB - 1)), 64);
  if (total_hits > kMaxOwn) raise_flag(c.ctr, kFlagCapPerParticle);
  const bool fits = base + wtot <= c.gcap;
  if (!fits && lane == 63) {
    atomicMax(&c.ctr->need_group, base + wtot);
    raise_flag(c.ctr, kFlagCapContacts);
  }
  if (s < n && fits) {
    if (sub == 0) {
      cn.off[s] = first;
      cn.cnt[s] = slot_end - first;
    }
    for (int k0 = 0; k0 < mine; k0 += 4) {
      int tk[4], rk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) tk[u] = k0 + u < mine ? hits[wv][k0 + u][lane] : -1;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (k0 + u < mine) {
          cn.a[first + k0 + u] = s;
          cn.b[first + k0 + u] = tk[u];
          const int l = base + incl - mine + k0 + u;  // record within the group
          if (FUSED && l < kThreads) {
            rec_a[l] = (unsigned char)(s - bg);
            rec_b[l] = tk[u];
          }
        }
      }
      // the partner-list places of up to four pairs are reserved together
#pragma unroll
      for (int u = 0; u < 4; ++u) rk[u] = tk[u] >= 0 ? atomicAdd(&c.pcnt[tk[u]], 1) : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (tk[u] < 0) continue;
        if (rk[u] < kMaxRev)
          c.plist[(size_t)rk[u] * c.pstride + tk[u]] = make_int2(s, first + k0 + u);
        else
          raise_flag(c.ctr, kFlagCapPerParticle);
      }
    }
  }
  return tot;
}

template <int SUB>
__global__ __launch_bounds__(kThreads) void k_detect(Ctx c, State A, State B, Contacts cn,
                                                    int rebuilt) {
  __shared__ int hits[kThreads / 64][kMaxOwn][64];
  __shared__ double xdrift[kThreads];
  __shared__ double red[kThreads / 64];
  __shared__ int wtots[kThreads / 64];
  (void)detect_group<SUB, false>(c, A, B, cn, rebuilt, xcd_remap(blockIdx.x, gridDim.x), hits,
                                 xdrift, red, wtots, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// 6. contact forces and torques (Section 2.2, 2.3, 3.2), one lane per contact.
//    On steps that keep the cells with one search lane per slot, on grids
//    resident in one round, the search of section 5 and this law run in one
//    workgroup per slot group (k_detect_force); otherwise k_detect and
//    k_force are launched one after the other.
// ---------------------------------------------------------------------------
// Static/kinetic update of a vector friction mode m in {s, r}: rotate the old
// spring into the tangent plane keeping its length, f = -k u - c v, then keep
// and integrate the spring (|f| <= lim) or clip f and reset the spring.
template <typename RT>
__device__ __forceinline__ void friction_vec(const RT n[3], RT k, RT cdmp, RT lim, double dt,
                                             const RT vm[3], double u[3], RT f[3]) {
  const double ul = sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  if (ul > 0.0) {
    const double un = (u[0] * (double)n[0] + u[1] * (double)n[1]) + u[2] * (double)n[2];
    double up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) up[a] = u[a] - un * (double)n[a];
    const double upl = sqrt((up[0] * up[0] + up[1] * up[1]) + up[2] * up[2]);
    if (upl > 0.0) {
      const double sc = ul / upl;
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = up[a] * sc;
    } else {
      u[0] = u[1] = u[2] = 0.0;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = -k * (RT)u[a] - cdmp * vm[a];
  const RT fl = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
  if (fl <= lim) {
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = u[a] + dt * (double)vm[a];
  } else {
    const RT sc = lim / fl;
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = f[a] * sc;
    const double ik = 1.0 / (double)k;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = -((double)f[a] + (double)cdmp * (double)vm[a]) * ik;
  }
}

template <typename RT>
__device__ __forceinline__ void friction_scalar(RT k, RT cdmp, RT lim, double dt, RT vm, double* u,
                                                RT* f) {
  RT ft = -k * (RT)(*u) - cdmp * vm;
  if (fabs(ft) <= lim) {
    *u = *u + dt * (double)vm;
  } else {
    ft = ft > (RT)0 ? lim : -lim;
    *u = -((double)ft + (double)cdmp * (double)vm) / (double)k;
  }
  *f = ft;
}

__device__ __forceinline__ double sphere_mass(double rho, double R) {
  return (4.0 / 3.0) * kPi * rho * (R * R * R);
}

// Record of key (ki, kj) among the n contacts that the previous owner slot
// owned in the previous step (records b0 ..), or -1 if the pair was not in
// contact.  Keys are probed four at a time so that their loads overlap.
__device__ __forceinline__ int find_old(const Contacts& co, int b0, int n, int2 key) {
  for (int base = 0; base < n; base += 4) {
    int2 k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) k[u] = base + u < n ? co.key[b0 + base + u] : make_int2(-1, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u < n && k[u].x == key.x && k[u].y == key.y) return b0 + base + u;
  }
  return -1;
}

// The contact law over the cnt records of slot group grp (the lane's record
// of the first pass in ra, rb; ng: the group's previous record count).  The
// spring and result records of one pass are staged in LDS (st_spr, st_res)
// and written out as contiguous runs (per-lane 64- and 80-byte records
// written directly would make every store instruction scatter); okey and red
// are LDS for the previous keys and the contact counts.
template <typename RT>
__device__ __forceinline__ void force_group(const Ctx& c, const State& S, const Contacts& cur,
                                            const Contacts& old, const int rebuilt, const int grp,
                                            const int ra, const int rb, const int ng,
                                            const int cnt, double2* st_spr, double2* st_res,
                                            int2* okey, int (*red)[kThreads / 64]) {
  const int tid = (int)threadIdx.x;
  const int gbase = grp * c.gcap;
  if (tid == 0) cur.ng[grp] = cnt;
  int npp = 0, npw = 0;
  // The contact law of one record (body I carries the lower id): the updated
  // springs are staged in LDS at this lane's place, the forces and torques
  // returned in o.
  auto law = [&](const SimParams& P, const bool wall, const int m, const bool swap,
                 const double4 pi, const double4 pj, const double2 va0, const double2 va1,
                 const double2 va2, const double2 vb0, const double2 vb1, const double2 vb2,
                 double* us, double* ur, double ut, const int e, const int2 key, double* o) {
    const double Ri = pi.w, Rj = pj.w;
    double dx, dy, dz, d;
    const double delta = pair_gap(pi.x, pi.y, pi.z, Ri, pj.x, pj.y, pj.z, Rj, &dx, &dy, &dz, &d);
    const double invd = 1.0 / d;
    const RT nrm[3] = {(RT)(dx * invd), (RT)(dy * invd), (RT)(dz * invd)};
    const double ri = Ri - 0.5 * delta;
    const double mi = sphere_mass(P.rho, Ri);
    const double2 vi0 = swap ? vb0 : va0, vi1 = swap ? vb1 : va1, vi2 = swap ? vb2 : va2;
    const double vix = vi0.x, viy = vi0.y, viz = vi1.x;
    const double wix = vi1.y, wiy = vi2.x, wiz = vi2.y;
    double rj, Rs, ms, Es, Gs, cnf, csf, reff;
    double vrel[3], om[3];
    const double n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
    if (!wall) {
      const double2 vj0 = swap ? va0 : vb0, vj1 = swap ? va1 : vb1, vj2 = swap ? va2 : vb2;
      const double vjx = vj0.x, vjy = vj0.y, vjz = vj1.x;
      const double wjx = vj1.y, wjy = vj2.x, wjz = vj2.y;
      rj = Rj - 0.5 * delta;
      const double mj = sphere_mass(P.rho, Rj);
      // effective radius and mass 1/(1/a + 1/b) written as a b / (a + b)
      Rs = (Ri * Rj) / (Ri + Rj);
      ms = (mi * mj) / (mi + mj);
      cnf = P.cnf_pp;
      csf = P.csf_pp;
      Es = P.Es_pp;
      Gs = P.Gs_pp;
      reff = (ri * rj) / (ri + rj);
      // v = v_i - v_j + n x (r_i w_i + r_j w_j)
      const double rx = ri * wix + rj * wjx, ry = ri * wiy + rj * wjy, rz = ri * wiz + rj * wjz;
      vrel[0] = (vix - vjx) + (n1 * rz - n2 * ry);
      vrel[1] = (viy - vjy) + (n2 * rx - n0 * rz);
      vrel[2] = (viz - vjz) + (n0 * ry - n1 * rx);
      om[0] = wix - wjx;
      om[1] = wiy - wjy;
      om[2] = wiz - wjz;
    } else {
      rj = 0.0;
      Rs = Ri;
      ms = mi;
      cnf = P.cnf_pw;
      csf = P.csf_pw;
      Es = P.Es_pw;
      Gs = P.Gs_pw;
      reff = ri;
      double vw0 = 0.0, vw1 = 0.0, vw2 = 0.0;
      double sw0 = 0.0, sw1 = 0.0, sw2 = 0.0;
      if (P.moving) {  // wall material velocity at the contact point p + R_m n
        const double* mv = c.tri_mv + 9 * (size_t)m;
        sw0 = mv[0];
        sw1 = mv[1];
        sw2 = mv[2];
        const double px = (pj.x + Rj * n0) - mv[3];
        const double py = (pj.y + Rj * n1) - mv[4];
        const double pz = (pj.z + Rj * n2) - mv[5];
        vw0 = (sw1 * pz - sw2 * py) + mv[6];
        vw1 = (sw2 * px - sw0 * pz) + mv[7];
        vw2 = (sw0 * py - sw1 * px) + mv[8];
      }
      const double rx = ri * wix, ry = ri * wiy, rz = ri * wiz;
      vrel[0] = (vix - vw0) + (n1 * rz - n2 * ry);
      vrel[1] = (viy - vw1) + (n2 * rx - n0 * rz);
      vrel[2] = (viz - vw2) + (n0 * ry - n1 * rx);
      om[0] = wix - sw0;
      om[1] = wiy - sw1;
      om[2] = wiz - sw2;
    }
    // coefficients (Eq. ks, cn, cs; k_r = k_n, c_r = c_n, k_t = k_s, c_t = c_s)
    // with k_n = 4/3 E* a and k_s = 8 G* a: c_n = beta sqrt(20/3 E*) sqrt(m* a)
    // and c_s = beta sqrt(4/3 G*) sqrt(m* a), the constant factors per simulation
    const RT ac = (RT)sqrt(Rs * delta);
    const RT kn = (RT)(4.0 / 3.0) * (RT)Es * ac;
    const RT ks = (RT)8.0 * (RT)Gs * ac;
    const RT sm = sqrt((RT)ms * ac);
    const RT cn = (RT)cnf * sm;
    const RT cs = (RT)csf * sm;
    // relative velocities
    const RT v0 = (RT)vrel[0], v1 = (RT)vrel[1], v2 = (RT)vrel[2];
    const RT vnn = (v0 * nrm[0] + v1 * nrm[1]) + v2 * nrm[2];
    const RT vn[3] = {vnn * nrm[0], vnn * nrm[1], vnn * nrm[2]};
    const RT vs[3] = {v0 - vn[0], v1 - vn[1], v2 - vn[2]};
    const RT o0 = (RT)om[0], o1 = (RT)om[1], o2 = (RT)om[2];
    const RT re = (RT)reff;
    const RT vr[3] = {re * (o1 * nrm[2] - o2 * nrm[1]), re * (o2 * nrm[0] - o0 * nrm[2]),
                      re * (o0 * nrm[1] - o1 * nrm[0])};
    const RT vt = (RT)Rs * ((o0 * nrm[0] + o1 * nrm[1]) + o2 * nrm[2]);
    // normal force f_n = k_n delta n - c_n v_n
    const RT kd = kn * (RT)delta;
    const RT fn[3] = {kd * nrm[0] - cn * vn[0], kd * nrm[1] - cn * vn[1], kd * nrm[2] - cn * vn[2]};
    const RT fnl = sqrt((fn[0] * fn[0] + fn[1] * fn[1]) + fn[2] * fn[2]);
    RT fs[3], fr[3], ft;
    friction_vec<RT>(nrm, ks, cs, (RT)P.mu_s * fnl, P.dt, vs, us, fs);
    friction_vec<RT>(nrm, kn, cn, (RT)P.mu_r * fnl, P.dt, vr, ur, fr);
    friction_scalar<RT>(ks, cs, (RT)P.mu_t * fnl, P.dt, vt, &ut, &ft);
    cur.key[e] = key;
    {
      double2* r = st_spr + (kSpr / 2) * threadIdx.x;
      r[0] = make_double2(us[0], us[1]);
      r[1] = make_double2(us[2], ur[0]);
      r[2] = make_double2(ur[1], ur[2]);
      r[3] = make_double2(ut, 0.0);
    }
    // torques: tau_s = r_i f_s x n, tau_r = R* n x f_r, tau_t = f_t R* n;
    // body j: -f, r_j f_s x n - tau_r - tau_t (Eq. antisymm_*)
    const RT fsxn[3] = {fs[1] * nrm[2] - fs[2] * nrm[1], fs[2] * nrm[0] - fs[0] * nrm[2],
                        fs[0] * nrm[1] - fs[1] * nrm[0]};
    const RT rs = (RT)Rs;
    const RT tr[3] = {rs * (nrm[1] * fr[2] - nrm[2] * fr[1]), rs * (nrm[2] * fr[0] - nrm[0] * fr[2]),
                      rs * (nrm[0] * fr[1] - nrm[1] * fr[0])};
    const RT ftr = ft * rs;
    const RT rif = (RT)ri, rjf = (RT)rj;
    npp += wall ? 0 : 1;
    npw += wall ? 1 : 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double f = (double)fn[k] + (double)fs[k];
      const double ttr = (double)tr[k] + (double)(ftr * nrm[k]);
      const double ti = (double)(rif * fsxn[k]) + ttr;
      const double tj = wall ? 0.0 : (double)(rjf * fsxn[k]) - ttr;
      // per-contact results for the owner slot a and the partner b
      o[k] = swap ? -f : f;
      o[3 + k] = swap ? ti : tj;  // torque on the partner
      o[6 + k] = swap ? tj : ti;  // torque on the owner
    }
    o[9] = 0.0;
  };
  auto stage_res = [&](const double* o) {
    double2* r = st_res + (kRes / 2) * threadIdx.x;
#pragma unroll
    for (int k = 0; k < kRes / 2; ++k) r[k] = make_double2(o[2 * k], o[2 * k + 1]);
  };
  auto write_out = [&](const int base) {
    const int nrec = min(cnt - base, kThreads);
    double2* gs = reinterpret_cast<double2*>(cur.spr + (size_t)kSpr * (gbase + base));
    for (int k = tid; k < nrec * (kSpr / 2); k += kThreads) gs[k] = st_spr[k];
    double2* gr = reinterpret_cast<double2*>(c.res + (size_t)kRes * (gbase + base));
    for (int k = tid; k < nrec * (kRes / 2); k += kThreads) gr[k] = st_res[k];
  };
  if (!rebuilt && cnt <= kThreads) {
    // The slot order was kept and the group's records fit one pass: the
    // previous step's records owned by this group's slots are the previous
    // records of the same group range.  Their keys and springs (the first
    // 256) come to LDS in contiguous runs while the bodies are gathered, and
    // each contact finds its springs there (the owner is the lower slot, a
    // slot of this group).  Two rounds of dependent loads instead of four.
    // The previous springs are held in the result staging buffer, which the
    // law's results overwrite only after every lane has read its springs.
    const bool act = tid < cnt;
    const int on = min(ng, kThreads);
    if (tid < on) {
      okey[tid] = old.key[gbase + tid];
      const double2* r = reinterpret_cast<const double2*>(old.spr + (size_t)kSpr * (gbase + tid));
      double2* d = st_res + (kSpr / 2) * tid;
      d[0] = r[0];
      d[1] = r[1];
      d[2] = r[2];
      d[3] = r[3];
    }
    const int a = ra, b = rb;
    const bool wall = b < 0;
    const SimParams* Pp = c.sp;
    double4 pa = make_double4(0.0, 0.0, 0.0, 0.0), pb = pa;
    double2 va0 = make_double2(0.0, 0.0), va1 = va0, va2 = va0, vb0 = va0, vb1 = va0, vb2 = va0;
    int ida = 0, idb = 0, m = 0, off = 0, n_o = 0;
    if (act) {
      Pp = c.sp + (c.nsims == 1 ? 0 : c.sim_of[a]);
      pa = S.xr[a];
      ida = S.pid[a];
      off = old.off[a];  // the owner's previous segment
      n_o = old.cnt[a];
      const double2* va = reinterpret_cast<const double2*>(S.vw + 6 * (size_t)a);
      va0 = va[0];
      va1 = va[1];
      va2 = va[2];
      if (!wall) {
        pb = S.xr[b];
        idb = S.pid[b];
        const double2* vb = reinterpret_cast<const double2*>(S.vw + 6 * (size_t)b);
        vb0 = vb[0];
        vb1 = vb[1];
        vb2 = vb[2];
      } else {
        m = -1 - b;
        const double p[3] = {pa.x, pa.y, pa.z};
        double cp[3];
        closest_on_element(p, c.tri + 9 * m, c.tri_nv[m], cp);
        pb = make_double4(cp[0], cp[1], cp[2], c.rmesh[m]);
      }
    }
    __syncthreads();
    double us[3] = {0.0, 0.0, 0.0}, ur[3] = {0.0, 0.0, 0.0}, ut = 0.0;
    bool swap = false;
    int2 key = make_int2(0, 0);
    if (act) {
      swap = !wall && ida > idb;
      key = wall ? make_int2(ida, -(m - Pp->tri0)) : make_int2(swap ? idb : ida, swap ? ida : idb);
      const int rel = off - gbase;
      double2 r0 = make_double2(0.0, 0.0), r1 = r0, r2 = r0, r3 = r0;
      bool found = false;
      if (n_o > 0 && rel >= 0 && rel + n_o <= on) {
        for (int k = 0; k < n_o; ++k) {
          const int2 kk = okey[rel + k];
          if (kk.x == key.x && kk.y == key.y) {
            const double2* q = st_res + (kSpr / 2) * (rel + k);
            r0 = q[0];
            r1 = q[1];
            r2 = q[2];
            r3 = q[3];
            found = true;
            break;
          }
        }
      } else {
        const int eo = find_old(old, off, n_o, key);
        if (eo >= 0) {
          const double2* q = reinterpret_cast<const double2*>(old.spr + (size_t)kSpr * eo);
          r0 = q[0];
          r1 = q[1];
          r2 = q[2];
          r3 = q[3];
          found = true;
        }
      }
      if (found) {
        us[0] = r0.x;
        us[1] = r0.y;
        us[2] = r1.x;
        ur[0] = r1.y;
        ur[1] = r2.x;
        ur[2] = r2.y;
        ut = r3.x;
      }
    }
    double o[kRes];
    if (act)
      law(*Pp, wall, m, swap, swap ? pb : pa, swap ? pa : pb, va0, va1, va2, vb0, vb1, vb2, us, ur,
          ut, gbase + tid, key, o);
    __syncthreads();  // every lane has read its previous springs
    if (act) stage_res(o);
    __syncthreads();
    write_out(0);
  } else {
    // (previous slot, its previous contact segment, id): carried by the
    // reorder, or the slot itself when the order was kept
    auto origin = [&](int p) {
      return rebuilt ? c.os[p] : make_int4(p, old.off[p], old.cnt[p], S.pid[p]);
    };
    for (int base = 0; base < cnt; base += kThreads) {
      const int l = base + tid;
      if (l < cnt) {
        const int e = gbase + l;
        const int a = cur.a[e], b = cur.b[e];
        const bool wall = b < 0;
        const SimParams& P = c.sp[c.nsims == 1 ? 0 : c.sim_of[a]];
        // both bodies are gathered at once; the canonical orientation is then
        // chosen in registers
        const double4 pa = S.xr[a];
        const int4 oa = origin(a);
        const double2* va = reinterpret_cast<const double2*>(S.vw + 6 * (size_t)a);
        const double2 va0 = va[0], va1 = va[1], va2 = va[2];
        double4 pb;
        int4 ob = oa;
        double2 vb0 = make_double2(0.0, 0.0), vb1 = vb0, vb2 = vb0;
        int m = 0;
        if (!wall) {
          pb = S.xr[b];
          // with the order kept the owner is the lower slot, so only the
          // partner's id is needed
          ob = rebuilt ? c.os[b] : make_int4(b, 0, 0, S.pid[b]);
          const double2* vb = reinterpret_cast<const double2*>(S.vw + 6 * (size_t)b);
          vb0 = vb[0];
          vb1 = vb[1];
          vb2 = vb[2];
        } else {
          m = -1 - b;
          const double p[3] = {pa.x, pa.y, pa.z};
          double cp[3];
          closest_on_element(p, c.tri + 9 * m, c.tri_nv[m], cp);
          pb = make_double4(cp[0], cp[1], cp[2], c.rmesh[m]);
        }
        // canonical orientation: body I carries the lower id (the particle for walls)
        const int ida = oa.w, idb = ob.w;
        const bool swap = !wall && ida > idb;
        const double4 pi = swap ? pb : pa, pj = swap ? pa : pb;
        const int2 key = wall ? make_int2(ida, -(m - P.tri0))
                              : make_int2(swap ? idb : ida, swap ? ida : idb);
        // springs of the previous step (zero for a new contact), looked up among
        // the records of the previous owner: the lower previous slot of the two
        double us[3] = {0.0, 0.0, 0.0}, ur[3] = {0.0, 0.0, 0.0}, ut = 0.0;
        {
          const bool bown = !wall && ob.x < oa.x;
          const int eo = find_old(old, bown ? ob.y : oa.y, bown ? ob.z : oa.z, key);
          if (eo >= 0) {
            const double2* r = reinterpret_cast<const double2*>(old.spr + (size_t)kSpr * eo);
            const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
            us[0] = r0.x;
            us[1] = r0.y;
            us[2] = r1.x;
            ur[0] = r1.y;
            ur[1] = r2.x;
            ur[2] = r2.y;
            ut = r3.x;
          }
        }
        double o[kRes];
        law(P, wall, m, swap, pi, pj, va0, va1, va2, vb0, vb1, vb2, us, ur, ut, e, key, o);
        stage_res(o);
      }
      __syncthreads();
      write_out(base);
      __syncthreads();
    }
  }
  // contact counts of the group for the statistics (summed by the next step's
  // grid kernel or by the host)
  const int a = wave_sum_i32(npp), b = wave_sum_i32(npw);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ta = 0, tb = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ta += red[0][w];
      tb += red[1][w];
    }
    // running sums, one writer per group: adds without a return value, so
    // the kernel's end does not wait for a read
    atomicAdd(&c.gstat[2 * grp], (unsigned long long)ta);
    atomicAdd(&c.gstat[2 * grp + 1], (unsigned long long)tb);
  }
}

template <typename RT>
__global__ __launch_bounds__(kThreads, 4) void k_force(Ctx c, State A, State B, Contacts cur,
                                                      Contacts old, int rebuilt) {
  const State S = rebuilt ? B : A;
  const int tid = (int)threadIdx.x;
  // one workgroup per slot group (on grids of one round, consecutive groups
  // share an XCD and its L2)
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  const int gbase = grp * c.gcap;
  // loads that depend on nothing else, issued together: this lane's record
  // of the first pass, the group's record count and, when the slot order was
  // kept, the group's previous record count
  int ra = 0, rb = 0;
  if (tid < c.gcap) {
    ra = cur.a[gbase + tid];
    rb = cur.b[gbase + tid];
  }
  const int ng = rebuilt ? 0 : old.ng[grp];
  const int cnt = min(c.gcnt[grp], c.gcap);
  // (the failure flag is examined once these loads are in flight; the
  // records are only followed after it)
  if (c.ctr->flags) return;
  __shared__ double2 st_spr[kThreads * kSpr / 2];
  __shared__ double2 st_res[kThreads * kRes / 2];
  __shared__ int2 okey[kThreads];
  __shared__ int red[2][kThreads / 64];
  force_group<RT>(c, S, cur, old, rebuilt, grp, ra, rb, ng, cnt, st_spr, st_res, okey, red);
}

// The search and the contact law of one slot group in one workgroup, for
// steps that keep the cells with one search lane per slot: the group's
// records reach the law through LDS (no second launch, no reload of the
// records), and the law's staging reuses the search's LDS (hit lists, drift
// reach), which is dead once the records are written.
template <typename RT>
__global__ __launch_bounds__(kThreads, 4) void k_detect_force(Ctx c, State A, State B,
                                                             Contacts cn, Contacts old) {
  constexpr int kHits2 = (kThreads / 64) * kMaxOwn * 64 * (int)sizeof(int) / 16;
  constexpr int kSearch2 = kHits2 + kThreads * (int)sizeof(double) / 16;
  constexpr int kLaw2 = kThreads * (kSpr + kRes) / 2;
  __shared__ double2 pool[kLaw2 > kSearch2 ? kLaw2 : kSearch2];
  __shared__ int2 okey[kThreads];
  __shared__ int rec_b[kThreads];
  __shared__ unsigned char rec_a[kThreads];
  __shared__ double red_d[kThreads / 64];
  __shared__ int wtots[kThreads / 64];
  __shared__ int red_i[2][kThreads / 64];
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  const int ng = old.ng[grp];
  const int tot = detect_group<1, true>(c, A, B, cn, 0, grp,
                                        reinterpret_cast<int(*)[kMaxOwn][64]>(pool),
                                        reinterpret_cast<double*>(pool + kHits2), red_d, wtots,
                                        rec_a, rec_b);
  // no forces after a flagged failure, or when this group's records did not
  // fit (flagged by the search: the step is repeated with more room)
  if (tot < 0 || tot > c.gcap) return;
  __syncthreads();  // the records are in LDS and global memory; the hit lists are dead
  const int tid = (int)threadIdx.x;
  int ra = 0, rb = 0;
  if (tid < tot) {
    ra = grp * kThreads + rec_a[tid];
    rb = rec_b[tid];
  }
  force_group<RT>(c, A, cn, old, 0, grp, ra, rb, ng, tot, pool, pool + kThreads * kSpr / 2, okey,
                  red_i);
}

// ---------------------------------------------------------------------------
// 7. integration: gather the contact sums of each particle in a fixed order
//    (owned contacts in record order, then partner contacts by ascending
//    owner slot), then semi-implicit Euler (Eq. v, x), SPIRAL (Eq. spiral)
//    with the old angular velocity, then Eq. w; Stokes drag (Section 2.1)
// ---------------------------------------------------------------------------
// sin(x)/x and cos(x).  The rotation angles of one step are tiny (|x| of
// order 1e-5), where the Taylor polynomials below are exact to far below one
// rounding (first omitted terms x^8/9! and x^10/10!, < 1e-24 relative for
// |x| < 2^-8); larger angles use the library.
__device__ __forceinline__ void sinc_cos(double x, double* sx, double* cx) {
  if (fabs(x) < 0.00390625) {
    const double x2 = x * x;
    *sx = 1.0 - x2 * (1.0 / 6.0 - x2 * (1.0 / 120.0 - x2 * (1.0 / 5040.0)));
    *cx = 1.0 - x2 * (0.5 - x2 * (1.0 / 24.0 - x2 * (1.0 / 720.0 - x2 * (1.0 / 40320.0))));
  } else {
    double sn, cs;
    sincos(x, &sn, &cs);
    *sx = sn / x;
    *cx = cs;
  }
}

__device__ __forceinline__ void qmul(const double a[4], const double b[4], double o[4]) {
  const double s = a[0] * b[0] - ((a[1] * b[1] + a[2] * b[2]) + a[3] * b[3]);
  const double x = (a[0] * b[1] + b[0] * a[1]) + (a[2] * b[3] - a[3] * b[2]);
  const double y = (a[0] * b[2] + b[0] * a[2]) + (a[3] * b[1] - a[1] * b[3]);
  const double z = (a[0] * b[3] + b[0] * a[3]) + (a[1] * b[2] - a[2] * b[1]);
  o[0] = s;
  o[1] = x;
  o[2] = y;
  o[3] = z;
}

__global__ __launch_bounds__(kThreads) void k_integrate(Ctx c, State A, State B, Contacts cur,
                                                       int rebuilt) {
  // reads the step's state (the sorted copy B, or A when the order was
  // kept) and writes the new state to B
  const State S = rebuilt ? B : A;
  const int n = c.n;
  const int i0 = xcd_remap(blockIdx.x, gridDim.x) * kThreads;
  const int i = i0 + (int)threadIdx.x;
  // The particle's own state and contact counts are loaded before the
  // failure flag is examined (a step after a failed one exits here): these
  // loads do not depend on the step's outcome so far, and the flag's round
  // trip then overlaps them.
  int sim = 0, e0 = 0, ne = 0, pc = 0;
  double4 xr = make_double4(0.0, 0.0, 0.0, 0.0), q4 = xr;
  double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0;
  if (i < n) {
    sim = c.nsims == 1 ? 0 : c.sim_of[i];
    xr = S.xr[i];
    q4 = S.q[i];
    const double2* vw2 = reinterpret_cast<const double2*>(S.vw + 6 * (size_t)i);
    s0 = vw2[0];
    s1 = vw2[1];
    s2 = vw2[2];
    e0 = cur.off[i];
    ne = cur.cnt[i];
    pc = c.pcnt[i];
  }
  if (c.ctr->flags) return;
  // new states are staged in LDS and written out as contiguous runs
  __shared__ double2 st_x[kThreads * 2], st_v[kThreads * 3], st_q[kThreads * 2];
  bool drift = false;
  double ddrift = 0.0;
  if (i < n) {
  const double* res = c.res;
  const SimParams& P = c.sp[sim];
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
  {
    // the partner list is loaded first, so that its gathers and those of
    // the owned records are in flight together
    const int e1 = e0 + ne;
    const int m = min(pc, kMaxRev);
    c.pcnt[i] = 0;  // cleared for the next step's narrow phase
    auto pl = [&](int j) { return c.plist[(size_t)j * c.pstride + i]; };
    int ka[8], ke[8];
    if (m <= 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int2 v = j < m ? pl(j) : make_int2(0x7fffffff, -1);
        ka[j] = v.x;
        ke[j] = v.y;
      }
    }
    // owned contacts in record order, four records in flight: the force
    // (doubles 0..2) and the owner's torque (6..8)
    for (int e = e0; e < e1; e += 4) {
      double2 f[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2* r = reinterpret_cast<const double2*>(res + (size_t)kRes * (e + u < e1 ? e + u : e));
        f[u][0] = r[0];
        f[u][1] = r[1];
        f[u][2] = r[3];
        f[u][3] = r[4];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (e + u < e1) {
          F[0] += f[u][0].x;
          F[1] += f[u][0].y;
          F[2] += f[u][1].x;
          T[0] += f[u][2].x;
          T[1] += f[u][2].y;
          T[2] += f[u][3].x;
        }
      }
    }
    // contacts owned by others, in ascending owner slot (the partner lists
    // hold (owner slot, record); owners of one partner are distinct)
    if (m <= 8) {
      // sort with a fixed compare-exchange network
#define SDEM_CX(x, y)                                    \
  if (ka[y] < ka[x]) {                                  \
    const int ta = ka[x], te = ke[x];                   \
    ka[x] = ka[y];                                      \
    ke[x] = ke[y];                                      \
    ka[y] = ta;                                         \
    ke[y] = te;                                         \
  }
      SDEM_CX(0, 1) SDEM_CX(2, 3) SDEM_CX(4, 5) SDEM_CX(6, 7)
      SDEM_CX(0, 2) SDEM_CX(1, 3) SDEM_CX(4, 6) SDEM_CX(5, 7)
      SDEM_CX(1, 2) SDEM_CX(5, 6) SDEM_CX(0, 4) SDEM_CX(3, 7)
      SDEM_CX(1, 5) SDEM_CX(2, 6)
      SDEM_CX(1, 4) SDEM_CX(3, 6)
      SDEM_CX(2, 4) SDEM_CX(3, 5)
      SDEM_CX(3, 4)
#undef SDEM_CX
      // force on the owner and torque on the partner: the first six doubles
      // of a record, four records in flight
#pragma unroll
      for (int j0 = 0; j0 < 8; j0 += 4) {
        if (j0 >= m) break;
        double2 g[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (j0 + u < m) {
            const double2* r = reinterpret_cast<const double2*>(res + (size_t)kRes * ke[j0 + u]);
            g[u][0] = r[0];
            g[u][1] = r[1];
            g[u][2] = r[2];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (j0 + u < m) {
            F[0] -= g[u][0].x;
            F[1] -= g[u][0].y;
            F[2] -= g[u][1].x;
            T[0] += g[u][1].y;
            T[1] += g[u][2].x;
            T[2] += g[u][2].y;
          }
        }
      }
    } else {
      int last = -1;
      for (int it = 0; it < m; ++it) {  // ascending owner slot
        int best = -1, ba = 0x7fffffff;
        for (int j = 0; j < m; ++j) {
          const int2 v = pl(j);
          if (v.x > last && v.x < ba) {
            ba = v.x;
            best = v.y;
          }
        }
        if (best < 0) break;
        last = ba;
        const double* r = res + (size_t)kRes * best;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          F[k] -= r[k];
          T[k] += r[3 + k];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c.F[k * n + i] = F[k];
    c.T[k * n + i] = T[k];
  }
  const double R = xr.w;
  const double m = sphere_mass(P.rho, R);
  const double I = 0.4 * m * R * R;
  const double cd = 9.0 * P.eta / (2.0 * P.rho * R * R);
  const double gd = (10.0 / 3.0) * cd;
  const double dt = P.dt;
  double v[3] = {s0.x, s0.y, s1.x}, w[3] = {s1.y, s2.x, s2.y};
  double x[3] = {xr.x, xr.y, xr.z}, al[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = (F[k] / m + P.g[k]) - cd * v[k];
    al[k] = T[k] / I - gd * w[k];
    v[k] = v[k] + dt * a;
    x[k] = x[k] + dt * v[k];
  }
  double q[4] = {q4.x, q4.y, q4.z, q4.w};
  const double wl = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
  if (wl > 0.0) {
    // sin(phi)/|w| = (dt/2) sin(phi)/phi
    const double phi = 0.5 * dt * wl;
    double sc, cp;
    sinc_cos(phi, &sc, &cp);
    const double sp = (0.5 * dt) * sc;
    const double r[4] = {cp, sp * w[0], sp * w[1], sp * w[2]};
    double o[4];
    qmul(q, r, o);
    q[0] = o[0]; q[1] = o[1]; q[2] = o[2]; q[3] = o[3];
  }
  const double alen = sqrt((al[0] * al[0] + al[1] * al[1]) + al[2] * al[2]);
  if (alen > 0.0) {
    // sin(theta)/|alpha| = (dt/2)^2 sin(theta)/theta
    const double h2 = (0.5 * dt) * (0.5 * dt);
    const double th = h2 * alen;
    double sc, ct;
    sinc_cos(th, &sc, &ct);
    const double st = h2 * sc;
    const double r[4] = {ct, st * al[0], st * al[1], st * al[2]};
    double o[4];
    qmul(q, r, o);
    q[0] = o[0]; q[1] = o[1]; q[2] = o[2]; q[3] = o[3];
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[k] = w[k] + dt * al[k];
    ok = ok && isfinite(x[k]) && isfinite(v[k]) && isfinite(w[k]);
  }
  const int t = threadIdx.x;
  if (!rebuilt) {  // the kept order: carry the slot's id over to B
    B.pid[i] = A.pid[i];
  }
  if (c.skin_on) {  // drift from the binned centre, and whether beyond half the skin
    const double4 xb = c.xb[i];
    const double ex = x[0] - xb.x, ey = x[1] - xb.y, ez = x[2] - xb.z;
    const double d2 = (ex * ex + ey * ey) + ez * ez;
    ddrift = sqrt(d2) * (1.0 + 1e-12);
    drift = d2 > P.half_skin * P.half_skin;
  }
  st_x[2 * t] = make_double2(x[0], x[1]);
  st_x[2 * t + 1] = make_double2(x[2], R);
  st_v[3 * t] = make_double2(v[0], v[1]);
  st_v[3 * t + 1] = make_double2(v[2], w[0]);
  st_v[3 * t + 2] = make_double2(w[1], w[2]);
  st_q[2 * t] = make_double2(q[0], q[1]);
  st_q[2 * t + 1] = make_double2(q[2], q[3]);
  if (!ok) raise_flag(c.ctr, kFlagNonFinite);
  if ((i & (kGroup - 1)) == 0) c.gcnt[i >> kGroupShift] = 0;  // for the next narrow phase
  }
  // a wave where a particle drifted past half the skin records its largest
  // drift (read by the next step's narrow phase) and raises the flag
  if (i - (int)(threadIdx.x & 63) < n && __any(drift)) {
    wave_drift(c, i, i < n, ddrift);
    // one write per wave, and none once the flag is up (a single address)
    if ((threadIdx.x & 63) == 0 && !c.ctr->rebuild_next) atomicOr(&c.ctr->rebuild_next, 1);
  }
  __syncthreads();
  const int np = min(n - i0, kThreads);
  double2* gx = reinterpret_cast<double2*>(B.xr + i0);
  double2* gv = reinterpret_cast<double2*>(B.vw + 6 * (size_t)i0);
  double2* gq = reinterpret_cast<double2*>(B.q + i0);
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gx[k] = st_x[k];
  for (int k = threadIdx.x; k < 3 * np; k += kThreads) gv[k] = st_v[k];
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gq[k] = st_q[k];
}

// ---------------------------------------------------------------------------
// state transfer between the caller's SoA arrays and the packed slots
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_scatter_state(Ctx c, State S, double* x, double* v,
                                                            double* w, double* q, double* F,
                                                            double* T) {
  const int n = c.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int id = S.pid[i];
  const double4 p = S.xr[i];
  const double* vw = S.vw + 6 * (size_t)i;
  if (x) {
    x[id] = p.x;
    x[n + id] = p.y;
    x[2 * n + id] = p.z;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (v) v[k * n + id] = vw[k];
    if (w) w[k * n + id] = vw[3 + k];
    if (F) F[k * n + id] = c.F[k * n + i];
    if (T) T[k * n + id] = c.T[k * n + i];
  }
  if (q) {
    const double4 qq = S.q[i];
    q[id] = qq.x;
    q[n + id] = qq.y;
    q[2 * n + id] = qq.z;
    q[3 * n + id] = qq.w;
  }
}

// slot i <- caller's particle i (identity order); v, w, q may be null
__global__ __launch_bounds__(kThreads) void k_pack_state(Ctx c, State S, const double* x,
                                                         const double* v, const double* w,
                                                         const double* q, const double* R) {
  const int n = c.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  S.xr[i] = make_double4(x[i], x[n + i], x[2 * n + i], R[i]);
  double* vw = S.vw + 6 * (size_t)i;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vw[k] = v ? v[k * n + i] : 0.0;
    vw[3 + k] = w ? w[k * n + i] : 0.0;
  }
  S.q[i] = q ? make_double4(q[i], q[n + i], q[2 * n + i], q[3 * n + i])
             : make_double4(1.0, 0.0, 0.0, 0.0);
  S.pid[i] = i;
  c.os[i] = make_int4(i, 0, 0, i);
  c.xb[i] = make_double4(x[i], x[n + i], x[2 * n + i], 0.0);
  c.key[i] = 0;
  c.F[i] = c.F[n + i] = c.F[2 * n + i] = 0.0;
  c.T[i] = c.T[n + i] = c.T[2 * n + i] = 0.0;
}

__global__ void k_selftest(int64_t n, const double* in, const double* in2, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = sqrt(in[i]);
  out[n + i] = in[i] / in2[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int n, int t) { return n > 0 ? (n + t - 1) / t : 1; }

hipError_t launch_step(const Ctx& c, const State& A, const State& B, const Contacts& cold,
                       const Contacts& cnew, int precision, int rebuild, hipStream_t s,
                       hipEvent_t* ev) {
  // rebuild: sort the particles into fresh cells (A -> B); otherwise the
  // cells and the slot order of A are kept and only the narrow phase, the
  // forces and the integration (A -> B) run.  ev (optional): kEvents events,
  // the phase boundaries and the force kernel's own start/stop.
  const int nbp = blocks_for(c.n, kThreads);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (rebuild) {
    k_bbox_part<<<nbp, kThreads, 0, s>>>(c, A);
    k_grid<<<1, kGridThreads, 0, s>>>(c);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (rebuild) {
    k_keys<<<nbp, kThreads, 0, s>>>(c, A);
    if (c.cap_cells <= kScanSmall) {
      k_scan_small<<<1, kScanOne, 0, s>>>(c);
    } else {
      k_scan_reduce<<<kScanBlocks, kScanThreads, 0, s>>>(c);
      k_scan_top<<<1, kScanThreads, 0, s>>>(c);
      k_scan_down<<<kScanBlocks, kScanThreads, 0, s>>>(c);
    }
    k_scatter<<<nbp, kThreads, 0, s>>>(c);
    k_reorder<<<nbp, kThreads, 0, s>>>(c, A, B, cold);
  }
  if (c.any_moving) {
    k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 0, rebuild);
    (void)launch_mesh_bins(c, s);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  // the search and the contact law in one kernel (in the force phase)
  const bool fused = fused_search_and_law(c, rebuild);
  if (!fused) switch (c.detect_sub) {
    case 1: k_detect<1><<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, A, B, cnew, rebuild); break;
    case 2: k_detect<2><<<blocks_for(2 * c.n, kThreads), kThreads, 0, s>>>(c, A, B, cnew, rebuild); break;
    case 8: k_detect<8><<<blocks_for(8 * c.n, kThreads), kThreads, 0, s>>>(c, A, B, cnew, rebuild); break;
    default: k_detect<4><<<blocks_for(4 * c.n, kThreads), kThreads, 0, s>>>(c, A, B, cnew, rebuild); break;
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  if (fused && ev) {
    // profiled: the dispatch itself records start and stop of the kernel
    const dim3 grid(c.ngroups), block(kThreads);
    if (precision == SDEM_MIXED)
      hipExtLaunchKernelGGL(k_detect_force<float>, grid, block, 0, s, ev[kPhases + 1],
                            ev[kPhases + 2], 0, c, A, B, cnew, cold);
    else
      hipExtLaunchKernelGGL(k_detect_force<double>, grid, block, 0, s, ev[kPhases + 1],
                            ev[kPhases + 2], 0, c, A, B, cnew, cold);
  } else if (fused && precision == SDEM_MIXED) {
    k_detect_force<float><<<c.ngroups, kThreads, 0, s>>>(c, A, B, cnew, cold);
  } else if (fused) {
    k_detect_force<double><<<c.ngroups, kThreads, 0, s>>>(c, A, B, cnew, cold);
  } else if (ev) {
    // profiled: the dispatch itself records start and stop of the kernel
    if (precision == SDEM_MIXED)
      hipExtLaunchKernelGGL(k_force<float>, dim3(c.ngroups), dim3(kThreads), 0, s, ev[kPhases + 1],
                            ev[kPhases + 2], 0, c, A, B, cnew, cold, rebuild);
    else
      hipExtLaunchKernelGGL(k_force<double>, dim3(c.ngroups), dim3(kThreads), 0, s, ev[kPhases + 1],
                            ev[kPhases + 2], 0, c, A, B, cnew, cold, rebuild);
  } else if (precision == SDEM_MIXED) {
    k_force<float><<<c.ngroups, kThreads, 0, s>>>(c, A, B, cnew, cold, rebuild);
  } else {
    k_force<double><<<c.ngroups, kThreads, 0, s>>>(c, A, B, cnew, cold, rebuild);
  }
  if (ev) (void)hipEventRecord(ev[4], s);
  k_integrate<<<nbp, kThreads, 0, s>>>(c, A, B, cnew, rebuild);
  if (ev) (void)hipEventRecord(ev[5], s);
  return hipGetLastError();
}

hipError_t launch_mesh_now(const Ctx& c, hipStream_t s) {
  // a moving mesh at the time of the step about to start (the step counter
  // does not count it yet)
  if (c.any_moving && c.ntri > 0)
    k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 0, 0);
  return hipGetLastError();
}

hipError_t launch_bbox(const Ctx& c, const State& S, hipStream_t s) {
  if (c.n > 0) k_bbox_part<<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, S);
  return hipGetLastError();
}

hipError_t launch_scatter_state(const Ctx& c, const State& S, double* x, double* v, double* w,
                                double* q, double* F, double* T, hipStream_t s) {
  if (c.n > 0)
    k_scatter_state<<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, S, x, v, w, q, F, T);
  return hipGetLastError();
}

hipError_t launch_pack_state(const Ctx& c, const State& S, const double* x, const double* v,
                             const double* w, const double* q, const double* R, hipStream_t s) {
  if (c.n > 0)
    k_pack_state<<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, S, x, v, w, q, R);
  return hipGetLastError();
}

hipError_t launch_mesh_planes(const Ctx& c, hipStream_t s) {
  if (c.ntri > 0) k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 1, 0);
  return hipGetLastError();
}

hipError_t launch_mesh_bins(const Ctx& c, hipStream_t s) {
  if (c.ntri > 0 && c.nbins > 0) {
    k_bin_count<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c);
    k_bin_scan<<<1, kBinScanThreads, 0, s>>>(c);
    k_bin_fill<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c);
    k_bin_sort<<<blocks_for(c.nbins, kThreads), kThreads, 0, s>>>(c);
  }
  return hipGetLastError();
}

hipError_t launch_selftest(int64_t n, const double* in, const double* in2, double* out,
                           hipStream_t s) {
  if (n > 0)
    k_selftest<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, in, in2, out);
  return hipGetLastError();
}

}  // namespace sdem
