// HIP kernels of one DEM time step on gfx950 (MI355X).
//
// Steps that rebuild the cells: bounding box -> grid -> cell keys + arrival
// ranks -> scan of the cell counts -> scatter -> stable reorder of the state
// into cell order; then (every step) one kernel per tile of 256 slots: the
// narrow phase, the contact law with the springs carried over, each
// particle's sums in a fixed order and the integration, all in one
// workgroup (steps that keep the cells start with a one-workgroup kernel
// that counts the step and turns a measured drift into extra reach).
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
      }
    }
    // bricks of 2^bits cells per axis (bits = min(3, ceil(log2 dim))); the
    // cell table covers whole bricks
    for (int k = 0; k < 3; ++k) {
      int b = 0;
      while (b < kBrickBits && (1 << b) < g.dim[k]) ++b;
      g.bits[k] = b;
      g.nb[k] = (g.dim[k] + (1 << b) - 1) >> b;
      nc *= (long long)g.nb[k] << b;
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

// Key of cell (cx, cy, cz) of a simulation's grid: the brick (row order of
// bricks), then the cell within it with the coordinate bits interleaved
// (x, y, z from the lowest bit up, axes with fewer bits dropping out).
__device__ __forceinline__ int cell_key(const SimGrid& g, int cx, int cy, int cz) {
  const int bx = g.bits[0], by = g.bits[1], bz = g.bits[2];
  int local = 0, pos = 0;
#pragma unroll
  for (int b = 0; b < kBrickBits; ++b) {
    if (b < bx) local |= ((cx >> b) & 1) << pos++;
    if (b < by) local |= ((cy >> b) & 1) << pos++;
    if (b < bz) local |= ((cz >> b) & 1) << pos++;
  }
  const int brick = ((cz >> bz) * g.nb[1] + (cy >> by)) * g.nb[0] + (cx >> bx);
  return g.cell_off + (brick << (bx + by + bz)) + local;
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
  const int key = cell_key(g, cx, cy, cz);
  c.key_tmp[i] = key;
  c.rank[i] = atomicAdd(&c.cell_cnt[key], 1);
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

// Writes the staged records of slots d0 .. d0+np-1 as contiguous runs of
// 16-byte stores (per-lane 32- and 64-byte records written directly would
// make every store instruction scatter).
__device__ __forceinline__ void copy_out(const State& B, int d0, int np, const double4* st_x,
                                         const Aux* st_a, const double4* st_q) {
  double2* gx = reinterpret_cast<double2*>(B.xr + d0);
  double2* ga = reinterpret_cast<double2*>(B.a + d0);
  double2* gq = reinterpret_cast<double2*>(B.q + d0);
  const double2* lx = reinterpret_cast<const double2*>(st_x);
  const double2* la = reinterpret_cast<const double2*>(st_a);
  const double2* lq = reinterpret_cast<const double2*>(st_q);
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gx[k] = lx[k];
  for (int k = threadIdx.x; k < 4 * np; k += kThreads) ga[k] = la[k];
  for (int k = threadIdx.x; k < 2 * np; k += kThreads) gq[k] = lq[k];
}

// Slot p of the scatter holds a particle of cell k; its final slot is the
// cell start plus the number of the cell's particles that came from a lower
// previous slot, so the order within a cell is the previous order (stable and
// deterministic).  Moves the whole state record.
__global__ __launch_bounds__(kThreads) void k_reorder(Ctx c, State A, State B) {
  if (c.ctr->flags) return;
  // Thread d fills new slot d.  The scatter put the particles of each cell in
  // arrival order; slot d of cell k takes the particle whose previous slot
  // ranks d - cell_start[k] among them (stable order within a cell).  The
  // record travels whole; its previous slot is noted (its contact segment of
  // the previous step is already in it).
  const int d0 = blockIdx.x * kThreads;
  const int d = d0 + (int)threadIdx.x;
  __shared__ double4 st_x[kThreads], st_q[kThreads];
  __shared__ Aux st_a[kThreads];
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
    const double4 xr = A.xr[so];
    Aux a = A.a[so];
    c.xb[d] = make_double4(xr.x, xr.y, xr.z, 0.0);  // binned centre
    a.prev = so;
    st_x[threadIdx.x] = xr;
    st_a[threadIdx.x] = a;
    st_q[threadIdx.x] = A.q[so];
  }
  __syncthreads();
  const int np = min(c.n - d0, kThreads);
  copy_out(B, d0, np, st_x, st_a, st_q);
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
    if (P.frame_bins && m == P.tri0) {
      double* f = c.frame + 12 * (size_t)c.tri_sim[m];
      for (int k = 0; k < 12; ++k) f[k] = 0.0;
      f[2] = 1.0;
      f[3] = 1.0;
      for (int k = 0; k < 3; ++k) f[5 + k] = f[8 + k] = G.center[k];
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
    if (P.frame_bins && m == P.tri0) {  // the frame the bins are looked up in
      double* f = c.frame + 12 * (size_t)c.tri_sim[m];
      const double ang = wl * tm;
      f[0] = wl > 0.0 ? G.omega[0] / wl : 0.0;
      f[1] = wl > 0.0 ? G.omega[1] / wl : 0.0;
      f[2] = wl > 0.0 ? G.omega[2] / wl : 1.0;
      f[3] = wl > 0.0 ? cos(ang) : 1.0;
      f[4] = wl > 0.0 ? sin(ang) : 0.0;
      f[5] = G.center[0] + d[0];
      f[6] = G.center[1] + d[1];
      f[7] = G.center[2] + d[2];
      f[8] = G.center[0];
      f[9] = G.center[1];
      f[10] = G.center[2];
    }
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
  const SimParams& P = c.sp[c.tri_sim[m]];
  const double* t = (P.frame_bins ? c.tri_ref : c.tri) + 9 * m;
  const bool rect = c.tri_nv[m] == 4;
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
// 5. one time step of a tile of 256 consecutive slots, in one workgroup:
//    narrow phase (Section 3.3), contact law with the springs carried over
//    (Section 2.2, 2.3), per-particle sums (Section 3.2) and integration
//    (Eq. v, x, spiral, w; Stokes drag of Section 2.1).
//
//    Each lane searches for the contacts of its particle with walls, with
//    every neighbour outside its tile, and with the neighbours of its tile
//    whose pair it owns (slot_owns: about half of them, for every lane
//    alike).  Contacts are then sorted into
//      - owned: walls, partners in a higher slot outside the tile, and the
//        tile's pairs the particle owns: evaluated here, springs written here;
//      - cross: partners in a lower slot outside the tile: evaluated here as
//        well (the partner's tile evaluates the same pair, bit for bit, and
//        writes its springs), this tile keeps only its own side;
//      - references: the tile's pairs that the partner owns, which the
//        search skips: the partner's record gives this particle's side (the
//        owner counts it for the particle, then appends the record's index
//        to the particle's reference list; each list is then sorted).
//    So no contact result leaves the workgroup: every particle's force and
//    torque are complete in LDS, and the tile integrates its particles at
//    once.  Per particle the sum runs in a fixed order (pass by pass: owned
//    records, cross records, references, each in record order), so results
//    do not depend on scheduling.  The work list (up to kLdsRec records)
//    stays in LDS; springs and the next state are stored from registers.
// ---------------------------------------------------------------------------
// Double-precision reciprocal, quotient and square root for the contact law
// (not for the contact test, whose square root stays correctly rounded): the
// hardware estimate refined by Newton steps, within a few ulps, a fraction
// of the instructions of the correctly rounded forms.  Arguments are finite;
// the square root takes x >= 0 (0 gives 0).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ double fast_div(double a, double b) {
  const double r = fast_rcp(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ double fast_sqrt(double x) {
  if (!(x > 0.0)) return 0.0;
  // y ~ 1/sqrt(x); g ~ sqrt(x), h ~ 1/(2 sqrt(x)), two coupled Newton steps
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}
// the same for the arithmetic type of the law (float: the library's forms)
__device__ __forceinline__ double rt_sqrt(double x) { return fast_sqrt(x); }
__device__ __forceinline__ float rt_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double rt_div(double a, double b) { return fast_div(a, b); }
__device__ __forceinline__ float rt_div(float a, float b) { return a / b; }

// Static/kinetic update of a vector friction mode m in {s, r}: rotate the old
// spring into the tangent plane keeping its length, f = -k u - c v, then keep
// and integrate the spring (|f| <= lim) or clip f and reset the spring.
template <typename RT>
__device__ __forceinline__ void friction_vec(const RT n[3], RT k, RT cdmp, RT lim, double dt,
                                             const RT vm[3], double u[3], RT f[3]) {
  const double ul = fast_sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  if (ul > 0.0) {
    const double un = (u[0] * (double)n[0] + u[1] * (double)n[1]) + u[2] * (double)n[2];
    double up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) up[a] = u[a] - un * (double)n[a];
    const double upl = fast_sqrt((up[0] * up[0] + up[1] * up[1]) + up[2] * up[2]);
    if (upl > 0.0) {
      const double sc = fast_div(ul, upl);
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = up[a] * sc;
    } else {
      u[0] = u[1] = u[2] = 0.0;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = -k * (RT)u[a] - cdmp * vm[a];
  const RT fl = rt_sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
  if (fl <= lim) {
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = u[a] + dt * (double)vm[a];
  } else {
    const RT sc = rt_div(lim, fl);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = f[a] * sc;
    const double ik = fast_rcp((double)k);
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
    *u = fast_div(-((double)ft + (double)cdmp * (double)vm), (double)k);
  }
  *f = ft;
}

__device__ __forceinline__ double sphere_mass(double rho, double R) {
  return (4.0 / 3.0) * kPi * rho * (R * R * R);
}

// The contact law of one contact.  Body I (centre and radius pi, velocity and
// spin vi) carries the lower persistent id, or is the particle of a wall
// contact; body J is the other particle, or for a wall the closest point of
// element m (pj.xyz) and the element radius (pj.w).  The springs us, ur, ut
// (orientation of body I) come in as carried over and leave updated.  Out:
// o[0..2] force on I, o[3..5] torque on I, o[6..8] torque on J (the force on
// J is -o[0..2]; Section 3.2).
template <typename RT>
__device__ __forceinline__ void contact_law(const Ctx& c, const SimParams& P, const bool wall,
                                            const int m, const double4 pi, const double4 pj,
                                            const double2 vi0, const double2 vi1,
                                            const double2 vi2, const double2 vj0,
                                            const double2 vj1, const double2 vj2, double us[3],
                                            double ur[3], double* ut, double o[9]) {
  const double Ri = pi.w, Rj = pj.w;
  double dx, dy, dz, d;
  const double delta = pair_gap(pi.x, pi.y, pi.z, Ri, pj.x, pj.y, pj.z, Rj, &dx, &dy, &dz, &d);
  const double invd = fast_rcp(d);
  const RT nrm[3] = {(RT)(dx * invd), (RT)(dy * invd), (RT)(dz * invd)};
  const double ri = Ri - 0.5 * delta;
  const double mi = sphere_mass(P.rho, Ri);
  const double vix = vi0.x, viy = vi0.y, viz = vi1.x;
  const double wix = vi1.y, wiy = vi2.x, wiz = vi2.y;
  double rj, Rs, ms, Es, Gs, cnf, csf, reff;
  double vrel[3], om[3];
  const double n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
  if (!wall) {
    const double vjx = vj0.x, vjy = vj0.y, vjz = vj1.x;
    const double wjx = vj1.y, wjy = vj2.x, wjz = vj2.y;
    rj = Rj - 0.5 * delta;
    const double mj = sphere_mass(P.rho, Rj);
    // effective radius and mass 1/(1/a + 1/b) written as a b / (a + b)
    Rs = fast_div(Ri * Rj, Ri + Rj);
    ms = fast_div(mi * mj, mi + mj);
    cnf = P.cnf_pp;
    csf = P.csf_pp;
    Es = P.Es_pp;
    Gs = P.Gs_pp;
    reff = fast_div(ri * rj, ri + rj);
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
  const RT ac = (RT)fast_sqrt(Rs * delta);
  const RT kn = (RT)(4.0 / 3.0) * (RT)Es * ac;
  const RT ks = (RT)8.0 * (RT)Gs * ac;
  const RT sm = rt_sqrt((RT)ms * ac);
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
  const RT fnl = rt_sqrt((fn[0] * fn[0] + fn[1] * fn[1]) + fn[2] * fn[2]);
  RT fs[3], fr[3], ft;
  friction_vec<RT>(nrm, ks, cs, (RT)P.mu_s * fnl, P.dt, vs, us, fs);
  friction_vec<RT>(nrm, kn, cn, (RT)P.mu_r * fnl, P.dt, vr, ur, fr);
  friction_scalar<RT>(ks, cs, (RT)P.mu_t * fnl, P.dt, vt, ut, &ft);
  // torques: tau_s = r_i f_s x n, tau_r = R* n x f_r, tau_t = f_t R* n;
  // body j: -f, r_j f_s x n - tau_r - tau_t (Eq. antisymm_*)
  const RT fsxn[3] = {fs[1] * nrm[2] - fs[2] * nrm[1], fs[2] * nrm[0] - fs[0] * nrm[2],
                      fs[0] * nrm[1] - fs[1] * nrm[0]};
  const RT rs = (RT)Rs;
  const RT tr[3] = {rs * (nrm[1] * fr[2] - nrm[2] * fr[1]), rs * (nrm[2] * fr[0] - nrm[0] * fr[2]),
                    rs * (nrm[0] * fr[1] - nrm[1] * fr[0])};
  const RT ftr = ft * rs;
  const RT rif = (RT)ri, rjf = (RT)rj;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ttr = (double)tr[k] + (double)(ftr * nrm[k]);
    o[k] = (double)fn[k] + (double)fs[k];
    o[3 + k] = (double)(rif * fsxn[k]) + ttr;
    o[6 + k] = wall ? 0.0 : (double)(rjf * fsxn[k]) - ttr;
  }
}

// A contact's springs between steps: the FP64 path keeps them as seven
// doubles in a 64-byte record; the mixed path rounds them to seven floats in
// a 32-byte record (the same buffer, read as floats), which halves the
// spring traffic.  Both update them in double within a step.
struct SpringF {
  float4 g0 = make_float4(0.f, 0.f, 0.f, 0.f), g1 = g0;
  __device__ __forceinline__ void load(const double* spr, int e) {
    const float4* q = reinterpret_cast<const float4*>(spr) + 2 * (size_t)e;
    g0 = q[0];
    g1 = q[1];
  }
  __device__ __forceinline__ void get(double us[3], double ur[3], double* ut) const {
    us[0] = g0.x;
    us[1] = g0.y;
    us[2] = g0.z;
    ur[0] = g0.w;
    ur[1] = g1.x;
    ur[2] = g1.y;
    *ut = g1.z;
  }
  __device__ __forceinline__ static void store(double* spr, int e, const double us[3],
                                               const double ur[3], double ut) {
    float4* q = reinterpret_cast<float4*>(spr) + 2 * (size_t)e;
    q[0] = make_float4((float)us[0], (float)us[1], (float)us[2], (float)ur[0]);
    q[1] = make_float4((float)ur[1], (float)ur[2], (float)ut, 0.f);
  }
};

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

// Block-wide exclusive scan of three counters at once (one value each per
// lane, lanes in slot order); returns the totals.  w3: LDS [waves][3].
__device__ __forceinline__ void block_scan3(int a, int b, int d, int* ea, int* eb, int* ed,
                                            int* ta, int* tb, int* td, int (*w3)[3]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int ia = a, ib = b, id = d;
  for (int o = 1; o < 64; o <<= 1) {
    const int ya = __shfl_up(ia, o, 64), yb = __shfl_up(ib, o, 64), yd = __shfl_up(id, o, 64);
    if (lane >= o) {
      ia += ya;
      ib += yb;
      id += yd;
    }
  }
  if (lane == 63) {
    w3[wv][0] = ia;
    w3[wv][1] = ib;
    w3[wv][2] = id;
  }
  __syncthreads();
  int pa = 0, pb = 0, pd = 0, sa = 0, sb = 0, sd = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wv) {
      pa += w3[w][0];
      pb += w3[w][1];
      pd += w3[w][2];
    }
    sa += w3[w][0];
    sb += w3[w][1];
    sd += w3[w][2];
  }
  *ea = pa + ia - a;
  *eb = pb + ib - b;
  *ed = pd + id - d;
  *ta = sa;
  *tb = sb;
  *td = sd;
}

// LDS of the step kernel.  The search's hit lists and the law's per-pass
// results share one pool.  Three workgroups fit a CU only while the whole
// stays below about 53.5 KB (54,112 bytes measured two per CU; now 51,296).
struct StepLds {
  union {
    int hits[kThreads / 64][kHit][64];
    struct {
      // force on I, torque on I, torque on J (and a pad: 16-byte rows)
      double2 res[kThreads][5];
    } law;
  } pool;
  int2 rec[kLdsRec];       // work list: (lane, partner)
  int ref[kLdsRef];        // references: partner slot, then the owner's record
  int ooff[kThreads];      // first owned record of each lane
  int roff[kThreads];      // each lane's reference count, then the next free place in its list
  int2 pseg[kThreads];     // each lane's owned records in the previous step (first, count)
  int w3[kThreads / 64][3];
  int cnt2[2][kThreads / 64];
  int flags;
};

// Opens a step that keeps the cells: counts it, and if the previous step saw
// a particle drift past half the skin, turns that into this step's extra
// reach per simulation (largest drift of its particles beyond half the skin,
// from the per-wave partials).  The step kernel reads what this writes; its
// own integration raises the flag for the next step.
constexpr int kBeginThreads = 1024;
__global__ __launch_bounds__(kBeginThreads) void k_begin(Ctx c) {
  if (c.ctr->flags) return;
  __shared__ int go;
  __shared__ double red[kBeginThreads / 64];
  if (threadIdx.x == 0) {
    c.ctr->steps += 1ull;
    const int d = c.ctr->rebuild_next;
    c.ctr->drift_now = d;
    c.ctr->rebuild_next = 0;
    if (d) c.ctr->drift_steps += 1ull;
    go = d;
  }
  __syncthreads();
  if (!go) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int sm = 0; sm < c.nsims; ++sm) {
    double dmax = 0.0;
    for (int q = c.chunk0[sm] + (int)threadIdx.x; q < c.chunk0[sm + 1]; q += kBeginThreads)
      dmax = fmax(dmax, c.part[kPart * q + 6]);
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    if (lane == 0) red[wv] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = red[0];
      for (int w = 1; w < kBeginThreads / 64; ++w) m = fmax(m, red[w]);
      const double ex = m - c.sp[sm].half_skin;
      c.xtra[sm] = ex > 0.0 ? ex * (1.0 + 1e-6) : 0.0;
    }
    __syncthreads();
  }
}

// One time step of the tile of slot group blockIdx (remapped per XCD): S is
// the state at the start of the step (the sorted copy on a step that rebuilt
// the cells), D receives the next state; cn the contacts of this step, old
// those of the previous step.
template <typename RT>
__global__ __launch_bounds__(kThreads, 3) void k_step(Ctx c, State S, State D, Contacts cn,
                                                     Contacts old, int rebuilt) {
  __shared__ StepLds L;
  const int n = c.n;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  const int base = grp * kThreads;
  const int s = base + tid;
  const bool valid = s < n;
  // The own centre, simulation and candidate list head are loaded before the
  // failure flag is examined (a step after a failed one exits there): none
  // depends on the step's outcome so far.  List entries are only followed
  // within the recorded count.
  int sim = 0, vcnt0 = -1, vraw[4] = {s, s, s, s};
  double4 ps = make_double4(0.0, 0.0, 0.0, 0.0);
  int2 pseg = make_int2(0, 0);
  if (valid) {
    sim = c.nsims == 1 ? 0 : c.sim_of[s];
    ps = S.xr[s];
    pseg = *reinterpret_cast<const int2*>(&S.a[s].off);
    if (c.skin_on && !rebuilt) {
      vcnt0 = c.vcnt[s];
#pragma unroll
      for (int u = 0; u < 4; ++u) vraw[u] = c.vlist[(size_t)u * c.vstride + s];
    }
  }
  if (tid == 0) L.flags = c.ctr->flags;
  L.roff[tid] = 0;  // references of each particle, counted by their owners
  __syncthreads();
  if (L.flags) return;  // the whole workgroup leaves together
  // If a particle drifted past half the skin since the cells were built (seen
  // by the previous step), every search of this step reaches by the excess
  // of its simulation further (k_begin)
  const bool drifted = !rebuilt && c.skin_on && c.ctr->drift_now;

  // ---- narrow phase: every contact of particle s, except those with a slot
  // of its own tile that owns the pair (slot_owns): that partner finds it
  // and hands it to s as a reference -------------------------------------------
  const int spill_cap = c.hit_cap - kHit;
  int nh = 0;
  auto put = [&](int t) {
    if (nh < kHit)
      L.pool.hits[wv][nh][lane] = t;
    else if (nh < c.hit_cap)
      c.spill[(size_t)s * spill_cap + (nh - kHit)] = t;
    ++nh;
  };
  auto hit = [&](int k) -> int {
    return k < kHit ? L.pool.hits[wv][k][lane] : c.spill[(size_t)s * spill_cap + (k - kHit)];
  };
  if (valid) {
    const double extra = drifted ? c.xtra[sim] : 0.0;
    const double xs = ps.x, ys = ps.y, zs = ps.z, Rs = ps.w;
    // Between rebuilds, with no drift past half the skin in this simulation,
    // the candidates recorded at the last rebuild suffice: every particle
    // within R_s + R_t + 2 (half skin) of x_s then, and (static meshes) every
    // element within R_s + R_m + half skin.
    const double hsk = c.sp[sim].half_skin;
    const bool listed = c.skin_on && !rebuilt && extra == 0.0;
    const bool record = c.skin_on && rebuilt;
    const bool tri_listed = !c.sp[sim].moving;
    auto vl = [&](int k) -> int& { return c.vlist[(size_t)k * c.vstride + s]; };
    const int nlist = listed ? vcnt0 : -1;
    int ncand = 0;
    auto test_wall = [&](int m) {
      const double p[3] = {xs, ys, zs};
      double cp[3];
      closest_on_element(p, c.tri + 9 * m, c.tri_nv[m], cp);
      double dx, dy, dz, d;
      const double delta = pair_gap(xs, ys, zs, Rs, cp[0], cp[1], cp[2], c.rmesh[m], &dx, &dy, &dz, &d);
      if (delta >= 0.0) put(-1 - m);
      return d;
    };
    auto test = [&](int t, const double4& pt) {
      const double ex = xs - pt.x, ey = ys - pt.y, ez = zs - pt.z;
      const double sr = Rs + pt.w;
      // cheap conservative reject before the exactly rounded test
      if ((ex * ex + ey * ey) + ez * ez > sr * sr * (1.0 + 1e-9)) return;
      double dx, dy, dz, d;
      const double delta = pair_gap(xs, ys, zs, Rs, pt.x, pt.y, pt.z, pt.w, &dx, &dy, &dz, &d);
      if (delta >= 0.0) put(t);
    };
    // ---- mesh elements listed in the bin of x_s (unless the list holds them)
    if (!(nlist >= 0 && tri_listed)) {
      int k0 = 0, k1 = 0;
      if (c.sp[sim].ntri > 0) {
        const MeshGrid G = c.mg[sim];
        double bx = xs, by = ys, bz = zs;
        if (c.sp[sim].frame_bins) {
          // the mesh moved as one rigid body since t = 0: its bins hold the
          // elements where they were then, so look up the particle moved back
          // (turned by minus the angle about the moved axis, centre back)
          const double* f = c.frame + 12 * (size_t)sim;
          const double rx = xs - f[5], ry = ys - f[6], rz = zs - f[7];
          const double kx = f[0], ky = f[1], kz = f[2], co = f[3], si = f[4];
          const double cx = ky * rz - kz * ry, cy = kz * rx - kx * rz, cz = kx * ry - ky * rx;
          const double kd = (kx * rx + ky * ry) + kz * rz;
          bx = f[8] + ((rx * co - cx * si) + kx * kd * (1.0 - co));
          by = f[9] + ((ry * co - cy * si) + ky * kd * (1.0 - co));
          bz = f[10] + ((rz * co - cz * si) + kz * kd * (1.0 - co));
        }
        const double fx = (bx - G.lo[0]) * G.inv_h, fy = (by - G.lo[1]) * G.inv_h,
                     fz = (bz - G.lo[2]) * G.inv_h;
        if (fx >= 0.0 && fy >= 0.0 && fz >= 0.0 && fx < (double)G.dim[0] &&
            fy < (double)G.dim[1] && fz < (double)G.dim[2]) {
          const int b = G.off + ((int)fz * G.dim[1] + (int)fy) * G.dim[0] + (int)fx;
          k0 = c.bin_start[b];
          k1 = c.bin_start[b + 1];
        }
      }
      const bool rec_tri = record && tri_listed;
      for (int k = k0; k < k1; ++k) {
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
    if (nlist >= 0) {
      // ---- particles (and listed elements) of the candidate list: four per
      // iteration; the next four slots are loaded while these are tested
      // (slots past the list read the own slot)
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
      // ---- cells: every cell within reach of x_s (all neighbours), row by
      // row, each row trimmed to the cells within reach of x_s given its
      // (y, z) distance (in cell units with margins far above rounding, so
      // the search only ever widens).  A rebuild looks twice as far to record
      // the candidates; a kept step reaches by the drift allowed since.
      const SimGrid gr = c.sg[sim];
      const double hs = record ? 2.0 * hsk : hsk + extra;
      const double reach = ((Rs + c.sp[sim].rmax) + hs) * (1.0 + 1e-9);
      const double rc = reach * gr.inv_h * (1.0 + 1e-9) + 1e-6;  // in cells
      const double fx = (xs - gr.lo[0]) * gr.inv_h, fy = (ys - gr.lo[1]) * gr.inv_h,
                   fz = (zs - gr.lo[2]) * gr.inv_h;
      const int z0 = cell_coord(zs - reach, gr.lo[2], gr.inv_h, gr.dim[2]);
      const int z1 = cell_coord(zs + reach, gr.lo[2], gr.inv_h, gr.dim[2]);
      const int y0 = cell_coord(ys - reach, gr.lo[1], gr.inv_h, gr.dim[1]);
      const int y1 = cell_coord(ys + reach, gr.lo[1], gr.inv_h, gr.dim[1]);
      // The cells of the box one after another, z then y then x; the slot
      // range of the next cell is loaded while the candidates of this one
      // are tested, and a cell whose key follows the previous one (x pairs
      // of a brick) starts where that one ended.
      int cz = z0, cy = y0 - 1, cx = 0, xend = -1;
      auto next_cell = [&]() -> int {
        for (;;) {
          if (cx < xend) {
            ++cx;
            return cell_key(gr, cx, cy, cz);
          }
          if (++cy > y1) {
            cy = y0;
            ++cz;
          }
          if (cz > z1) return -1;
          const double dz = fmax(fmax((double)cz - fz, fz - (double)(cz + 1)) - 1e-6, 0.0);
          const double dy = fmax(fmax((double)cy - fy, fy - (double)(cy + 1)) - 1e-6, 0.0);
          const double d2 = dy * dy + dz * dz;
          if (d2 > rc * rc) continue;
          const double xr = sqrt(rc * rc - d2) * (1.0 + 1e-9) + 1e-6;
          const int xa = max(0, (int)floor(fx - xr)), xb = min(gr.dim[0] - 1, (int)floor(fx + xr));
          if (xb < xa) continue;
          cx = xa;
          xend = xb;
          return cell_key(gr, cx, cy, cz);
        }
      };
      int key = next_cell();
      int c0 = 0, c1 = 0;
      if (key >= 0) {
        c0 = c.cell_start[key];
        c1 = c.cell_start[key + 1];
      }
      while (key >= 0) {
        const int t0 = c0, t1 = c1;
        const int kn = next_cell();
        if (kn >= 0) {
          c0 = kn == key + 1 ? t1 : c.cell_start[kn];
          c1 = c.cell_start[kn + 1];
        }
        key = kn;
        for (int t = t0; t < t1; t += 4) {
          double4 pt[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pt[u] = S.xr[t + u < t1 ? t + u : t];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int tu = t + u;
            if (tu >= t1) break;
            // itself, or a pair of the tile that the other side owns
            if (tu == s || (tu >= base && tu - base < kThreads && !slot_owns(s, tu))) continue;
            if (record) {
              const double ex = xs - pt[u].x, ey = ys - pt[u].y, ez = zs - pt[u].z;
              const double sr = (Rs + pt[u].w) + 2.0 * hsk;
              if ((ex * ex + ey * ey) + ez * ez <= sr * sr * (1.0 + 1e-9)) {
                if (ncand < kCand) vl(ncand) = tu;
                ++ncand;
              }
            }
            test(tu, pt[u]);
          }
        }
      }
    }
    if (record) c.vcnt[s] = ncand <= kCand ? ncand : -1;  // -1: search the cells
  }
  // ---- work lists: owned, cross and referenced contacts of the tile --------
  // Every pair of the tile found is owned; a particle's references are the
  // owned records of other lanes whose partner it is: their owners count them.
  const int nk = nh < c.hit_cap ? nh : c.hit_cap;
  int no = 0, nx = 0;
  for (int k = 0; k < nk; ++k) {
    const int t = hit(k);
    if (t < 0 || t >= base) {
      ++no;
      if (t >= base && t - base < kThreads) atomicAdd(&L.roff[t - base], 1);
    } else {
      ++nx;
    }
  }
  __syncthreads();
  const int nr = L.roff[tid];
  int ooff, xoff, roff, To, Tx, Tr;
  block_scan3(no, nx, nr, &ooff, &xoff, &roff, &To, &Tx, &Tr, L.w3);
  const int gbase = grp * c.gcap;   // owned records (springs, keys)
  const int wbase = 2 * gbase;      // work list past the LDS
  const bool over_p = nh + nr > c.hit_cap;
  const bool over_g = To > c.gcap || To + Tx > 2 * c.gcap || Tr > kLdsRef + c.gcap;
  if (over_p) raise_flag(c.ctr, kFlagCapPerParticle);
  if (over_g && tid == 0) {
    atomicMax(&c.ctr->need_group, max(To, (To + Tx + 1) / 2));
    raise_flag(c.ctr, kFlagCapContacts);
  }
  // a tile whose lists do not fit stops here; the step is failed and repeated
  // by the caller with more room (no state of the step is kept)
  if (over_g) return;
  auto ref_at = [&](int q) -> int {
    return q < kLdsRef ? L.ref[q] : cn.ref[gbase + (q - kLdsRef)];
  };
  auto ref_set = [&](int q, int v) {
    if (q < kLdsRef)
      L.ref[q] = v;
    else
      cn.ref[gbase + (q - kLdsRef)] = v;
  };
  for (int j = 0; j < nr; ++j) ref_set(roff + j, -1);
  L.ooff[tid] = ooff;
  L.roff[tid] = roff;
  L.pseg[tid] = pseg;
  __syncthreads();
  {
    // owned and cross records; an owned record whose partner is a slot of
    // the tile is also that partner's reference (it lists the pair the other
    // way round), appended to the partner's list
    int jo = 0, jx = 0;
    for (int k = 0; k < nk; ++k) {
      const int t = hit(k);
      if (t < 0 || t >= base) {
        const int r = ooff + jo++;
        if (r < kLdsRec) L.rec[r] = make_int2(tid, t);
        else {
          cn.a[wbase + r] = tid;
          cn.b[wbase + r] = t;
        }
        if (t >= base && t - base < kThreads) {
          // (the same appends were counted above, so q stays within the
          // partner's list)
          const int q = atomicAdd(&L.roff[t - base], 1);
          if (q < Tr) ref_set(q, r);
        }
      } else {
        const int r = To + xoff + jx++;
        if (r < kLdsRec) L.rec[r] = make_int2(tid, t);
        else {
          cn.a[wbase + r] = tid;
          cn.b[wbase + r] = t;
        }
      }
    }
  }
  if (valid) {
    cn.off[s] = gbase + ooff;
    cn.cnt[s] = no;
  }
  if (tid == 0) cn.ng[grp] = To;
  __syncthreads();
  auto rec_at = [&](int r) -> int2 {
    return r < kLdsRec ? L.rec[r] : make_int2(cn.a[wbase + r], cn.b[wbase + r]);
  };
  // the particle's references in ascending record order (each pass then
  // takes a run of them); they arrived in any order.  Up to eight (the usual
  // case) are sorted in registers by Batcher's odd-even merge network for
  // eight inputs (19 comparators), more by insertion in place.
  if (nr > 1 && nr <= 8 && roff + nr <= kLdsRef) {
    int v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = k < nr ? L.ref[roff + k] : INT_MAX;
    auto cs = [&](int a, int b) {
      const int lo = min(v[a], v[b]), hi = max(v[a], v[b]);
      v[a] = lo;
      v[b] = hi;
    };
    cs(0, 1); cs(2, 3); cs(4, 5); cs(6, 7);
    cs(0, 2); cs(1, 3); cs(4, 6); cs(5, 7);
    cs(1, 2); cs(5, 6);
    cs(0, 4); cs(1, 5); cs(2, 6); cs(3, 7);
    cs(2, 4); cs(3, 5);
    cs(1, 2); cs(3, 4); cs(5, 6);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < nr) L.ref[roff + k] = v[k];
  } else {
    for (int j = 1; j < nr; ++j) {
      const int v = ref_at(roff + j);
      int k = roff + j;
      for (; k > roff; --k) {
        const int prev = ref_at(k - 1);
        if (prev <= v) break;
        ref_set(k, prev);
      }
      ref_set(k, v);
    }
  }

  // ---- contact law, pass by pass over the work list ------------------------
  const int nrec = To + Tx;
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
  // (previous slot, its previous contact segment, id) of a particle, in its
  // record: noted by the reorder, or by the previous step when the order
  // was kept
  auto origin = [&](int p) {
    const int4 v = *reinterpret_cast<const int4*>(&S.a[p].pid);
    return make_int4(v.y, v.z, v.w, v.x);
  };
  int npp = 0, npw = 0;
  int jr = 0;  // the particle's next reference to sum
  for (int p0 = 0; p0 < nrec; p0 += kThreads) {
    __syncthreads();  // the pool's last use (hit lists, or the previous pass) is over
    const int r = p0 + tid;
    if (r < nrec) {
      const int2 rb = rec_at(r);
      const int a = base + rb.x, b = rb.y;
      const bool wall = b < 0;
      const SimParams& P = c.sp[c.nsims == 1 ? 0 : c.sim_of[a]];
      // both bodies are gathered at once; the canonical orientation is then
      // chosen in registers
      const double4 pa = S.xr[a];
      const int4 oa = origin(a);
      const double2 va0 = S.a[a].vw[0], va1 = S.a[a].vw[1], va2 = S.a[a].vw[2];
      double4 pb;
      int4 ob = oa;
      double2 vb0 = make_double2(0.0, 0.0), vb1 = vb0, vb2 = vb0;
      int m = 0;
      if (!wall) {
        pb = S.xr[b];
        ob = origin(b);
        vb0 = S.a[b].vw[0];
        vb1 = S.a[b].vw[1];
        vb2 = S.a[b].vw[2];
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
      const int2 key = wall ? make_int2(ida, -(m - P.tri0))
                            : make_int2(swap ? idb : ida, swap ? ida : idb);
      // springs of the previous step (zero for a new contact), looked up among
      // the records of the previous owner (slot_owns of the previous slots).
      // A particle's contacts come out of its search in the same order every
      // step (candidates in list order) unless some formed or ended, so the
      // previous record of its j-th owned contact is most often its j-th
      // previous record: that one (key and springs) is loaded with the bodies,
      // and the segment is searched only when its key differs.
      double us[3] = {0.0, 0.0, 0.0}, ur[3] = {0.0, 0.0, 0.0}, ut = 0.0;
      if constexpr (sizeof(RT) == sizeof(double)) {
        int2 kg = make_int2(-1, 0);
        double2 g0 = make_double2(0.0, 0.0), g1 = g0, g2 = g0, g3 = g0;
        int eg = -1;
        if (r < To) {
          const int j = r - L.ooff[rb.x];
          const int2 ps2 = L.pseg[rb.x];
          if (j < ps2.y) eg = ps2.x + j;
        }
        if (eg >= 0) {
          kg = old.key[eg];
          const double2* q = reinterpret_cast<const double2*>(old.spr + (size_t)kSpr * eg);
          g0 = q[0];
          g1 = q[1];
          g2 = q[2];
          g3 = q[3];
        }
        int eo = -1;
        if (eg >= 0 && kg.x == key.x && kg.y == key.y) {
          eo = eg;
        } else {
          const bool bown = !wall && slot_owns(ob.x, oa.x);
          eo = find_old(old, bown ? ob.y : oa.y, bown ? ob.z : oa.z, key);
          if (eo >= 0) {
            const double2* q = reinterpret_cast<const double2*>(old.spr + (size_t)kSpr * eo);
            g0 = q[0];
            g1 = q[1];
            g2 = q[2];
            g3 = q[3];
          }
        }
        if (eo >= 0) {
          us[0] = g0.x;
          us[1] = g0.y;
          us[2] = g1.x;
          ur[0] = g1.y;
          ur[1] = g2.x;
          ur[2] = g2.y;
          ut = g3.x;
        }
      } else {
        // the same lookup over the 32-byte float records of the mixed path
        int2 kg = make_int2(-1, 0);
        SpringF g;
        int eg = -1;
        if (r < To) {
          const int j = r - L.ooff[rb.x];
          const int2 ps2 = L.pseg[rb.x];
          if (j < ps2.y) eg = ps2.x + j;
        }
        if (eg >= 0) {
          kg = old.key[eg];
          g.load(old.spr, eg);
        }
        int eo = -1;
        if (eg >= 0 && kg.x == key.x && kg.y == key.y) {
          eo = eg;
        } else {
          const bool bown = !wall && slot_owns(ob.x, oa.x);
          eo = find_old(old, bown ? ob.y : oa.y, bown ? ob.z : oa.z, key);
          if (eo >= 0) g.load(old.spr, eo);
        }
        if (eo >= 0) g.get(us, ur, &ut);
      }
      // one call of the law for the whole wave: the canonical orientation is
      // chosen in registers (two calls behind a branch on swap would make a
      // wave whose lanes differ run both)
      double o[9];
      {
        const double4 pi = swap ? pb : pa, pj = swap ? pa : pb;
        const double2 vi0 = swap ? vb0 : va0, vi1 = swap ? vb1 : va1, vi2 = swap ? vb2 : va2;
        const double2 vj0 = swap ? va0 : vb0, vj1 = swap ? va1 : vb1, vj2 = swap ? va2 : vb2;
        contact_law<RT>(c, P, wall, m, pi, pj, vi0, vi1, vi2, vj0, vj1, vj2, us, ur, &ut, o);
      }
      // results by the tile's particle a (force on a, torque on a, torque on b)
      double ra[9];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ra[k] = swap ? -o[k] : o[k];
        ra[3 + k] = swap ? o[6 + k] : o[3 + k];
        ra[6 + k] = swap ? o[3 + k] : o[6 + k];
      }
      double2* rs = L.pool.law.res[tid];
      rs[0] = make_double2(ra[0], ra[1]);
      rs[1] = make_double2(ra[2], ra[3]);
      rs[2] = make_double2(ra[4], ra[5]);
      rs[3] = make_double2(ra[6], ra[7]);
      rs[4] = make_double2(ra[8], 0.0);
      if (r < To) {
        // the owned record's key and springs: consecutive lanes write
        // consecutive records
        if constexpr (sizeof(RT) == sizeof(double)) {
          double2* gs = reinterpret_cast<double2*>(cn.spr + (size_t)kSpr * (gbase + r));
          gs[0] = make_double2(us[0], us[1]);
          gs[1] = make_double2(us[2], ur[0]);
          gs[2] = make_double2(ur[1], ur[2]);
          gs[3] = make_double2(ut, 0.0);
        } else {
          SpringF::store(cn.spr, gbase + r, us, ur, ut);
        }
        cn.key[gbase + r] = key;
        npp += wall ? 0 : 1;
        npw += wall ? 1 : 0;
      }
    }
    __syncthreads();
    // the tile's particles take their sides of this pass's records
    if (valid) {
      const int p1 = p0 + kThreads;
      auto take = [&](int rr) {
        const double2* x = L.pool.law.res[rr - p0];
        const double2 a = x[0], b = x[1], d = x[2];
        F[0] += a.x; F[1] += a.y; F[2] += b.x;
        T[0] += b.y; T[1] += d.x; T[2] += d.y;
      };
      for (int rr = max(ooff, p0); rr < min(ooff + no, p1); ++rr) take(rr);
      const int x0 = To + xoff;
      for (int rr = max(x0, p0); rr < min(x0 + nx, p1); ++rr) take(rr);
      for (; jr < nr; ++jr) {
        const int rr = ref_at(roff + jr);
        if (rr >= p1) break;
        if (rr < p0) continue;  // (-1: no record found)
        const double2* x = L.pool.law.res[rr - p0];
        const double2 a = x[0], b = x[1], d = x[3], e = x[4];
        F[0] -= a.x; F[1] -= a.y; F[2] -= b.x;
        T[0] += d.x; T[1] += d.y; T[2] += e.x;
      }
    }
  }
  // contact counts of the tile for the statistics (running sums, one writer
  // per group)
  {
    const int a = wave_sum_i32(npp), b = wave_sum_i32(npw);
    if (lane == 0) {
      L.cnt2[0][wv] = a;
      L.cnt2[1][wv] = b;
    }
  }
  __syncthreads();  // also: the pool's law results are dead from here
  if (tid == 0) {
    int ta = 0, tb = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      ta += L.cnt2[0][w];
      tb += L.cnt2[1][w];
    }
    atomicAdd(&c.gstat[2 * grp], (unsigned long long)ta);
    atomicAdd(&c.gstat[2 * grp + 1], (unsigned long long)tb);
  }

  // ---- integration of the tile's particles ---------------------------------
  bool drift = false;
  double ddrift = 0.0;
  if (valid) {
    const SimParams& P = c.sp[sim];
    const double2 s0 = S.a[s].vw[0], s1 = S.a[s].vw[1], s2 = S.a[s].vw[2];
    const double4 q4 = S.q[s];
    const int pid = S.a[s].pid;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c.F[k * n + s] = F[k];
      c.T[k * n + s] = T[k];
    }
    const double R = ps.w;
    const double m = sphere_mass(P.rho, R);
    const double I = 0.4 * m * R * R;
    const double cd = 9.0 * P.eta / (2.0 * P.rho * R * R);
    const double gd = (10.0 / 3.0) * cd;
    const double dt = P.dt;
    double v[3] = {s0.x, s0.y, s1.x}, w[3] = {s1.y, s2.x, s2.y};
    double x[3] = {ps.x, ps.y, ps.z}, al[3];
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
      const double r4[4] = {cp, sp * w[0], sp * w[1], sp * w[2]};
      double o4[4];
      qmul(q, r4, o4);
      q[0] = o4[0]; q[1] = o4[1]; q[2] = o4[2]; q[3] = o4[3];
    }
    const double alen = sqrt((al[0] * al[0] + al[1] * al[1]) + al[2] * al[2]);
    if (alen > 0.0) {
      // sin(theta)/|alpha| = (dt/2)^2 sin(theta)/theta
      const double h2 = (0.5 * dt) * (0.5 * dt);
      const double th = h2 * alen;
      double sc, ct;
      sinc_cos(th, &sc, &ct);
      const double st = h2 * sc;
      const double r4[4] = {ct, st * al[0], st * al[1], st * al[2]};
      double o4[4];
      qmul(q, r4, o4);
      q[0] = o4[0]; q[1] = o4[1]; q[2] = o4[2]; q[3] = o4[3];
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      w[k] = w[k] + dt * al[k];
      ok = ok && isfinite(x[k]) && isfinite(v[k]) && isfinite(w[k]);
    }
    if (c.skin_on) {  // drift from the binned centre, and whether beyond half the skin
      const double4 xb = c.xb[s];
      const double ex = x[0] - xb.x, ey = x[1] - xb.y, ez = x[2] - xb.z;
      const double d2 = (ex * ex + ey * ey) + ez * ez;
      ddrift = sqrt(d2) * (1.0 + 1e-12);
      drift = d2 > P.half_skin * P.half_skin;
    }
    // the next state; consecutive lanes write consecutive slots.  The record
    // notes this order as the next step's previous one, and where the
    // particle's owned records are.
    D.xr[s] = make_double4(x[0], x[1], x[2], R);
    D.q[s] = make_double4(q[0], q[1], q[2], q[3]);
    Aux& o = D.a[s];
    o.vw[0] = make_double2(v[0], v[1]);
    o.vw[1] = make_double2(v[2], w[0]);
    o.vw[2] = make_double2(w[1], w[2]);
    *reinterpret_cast<int4*>(&o.pid) = make_int4(pid, s, gbase + ooff, no);
    if (!ok) raise_flag(c.ctr, kFlagNonFinite);
  }
  // a wave where a particle drifted past half the skin records its largest
  // drift (read by the next step's narrow phase) and raises the flag
  if (s - lane < n && __any(drift)) {
    wave_drift(c, s, valid, ddrift);
    // one write per wave, and none once the flag is up (a single address)
    if (lane == 0 && !c.ctr->rebuild_next) atomicOr(&c.ctr->rebuild_next, 1);
  }
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
  const Aux r = S.a[i];
  const double4 p = S.xr[i];
  const int id = r.pid;
  const double vw[6] = {r.vw[0].x, r.vw[0].y, r.vw[1].x, r.vw[1].y, r.vw[2].x, r.vw[2].y};
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
  Aux r;
  S.xr[i] = make_double4(x[i], x[n + i], x[2 * n + i], R[i]);
  double vw[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vw[k] = v ? v[k * n + i] : 0.0;
    vw[3 + k] = w ? w[k * n + i] : 0.0;
  }
  r.vw[0] = make_double2(vw[0], vw[1]);
  r.vw[1] = make_double2(vw[2], vw[3]);
  r.vw[2] = make_double2(vw[4], vw[5]);
  S.q[i] = q ? make_double4(q[i], q[n + i], q[2 * n + i], q[3 * n + i])
             : make_double4(1.0, 0.0, 0.0, 0.0);
  r.pid = i;
  r.prev = i;
  r.off = 0;
  r.cnt = 0;
  S.a[i] = r;
  c.xb[i] = make_double4(x[i], x[n + i], x[2 * n + i], 0.0);
  c.F[i] = c.F[n + i] = c.F[2 * n + i] = 0.0;
  c.T[i] = c.T[n + i] = c.T[2 * n + i] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_set_segments(Ctx c, State S, Contacts cn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  S.a[i].off = cn.off[i];
  S.a[i].cnt = cn.cnt[i];
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

hipError_t launch_step(const Ctx& c, const State& A, const State& B, const State& T,
                       const Contacts& cold, const Contacts& cnew, int precision, int rebuild,
                       hipStream_t s, hipEvent_t* ev) {
  // rebuild: sort the particles of A into fresh cells (copy T), then step
  // T -> B; otherwise the cells and the slot order of A are kept and the step
  // runs A -> B.  ev (optional): kEvents events, the phase boundaries and the
  // step kernel's own start/stop.
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
    k_reorder<<<nbp, kThreads, 0, s>>>(c, A, T);
  }
  if (c.any_moving) {
    k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 0, rebuild);
    if (c.rebin) (void)launch_mesh_bins(c, s);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  if (!rebuild) k_begin<<<1, kBeginThreads, 0, s>>>(c);
  if (ev) (void)hipEventRecord(ev[3], s);
  const State& S = rebuild ? T : A;
  const dim3 grid(c.ngroups), block(kThreads);
  if (ev) {
    // profiled: the dispatch itself records start and stop of the kernel
    if (precision == SDEM_MIXED)
      hipExtLaunchKernelGGL(k_step<float>, grid, block, 0, s, ev[kPhases + 1], ev[kPhases + 2], 0,
                            c, S, B, cnew, cold, rebuild);
    else
      hipExtLaunchKernelGGL(k_step<double>, grid, block, 0, s, ev[kPhases + 1], ev[kPhases + 2],
                            0, c, S, B, cnew, cold, rebuild);
  } else if (precision == SDEM_MIXED) {
    k_step<float><<<grid, block, 0, s>>>(c, S, B, cnew, cold, rebuild);
  } else {
    k_step<double><<<grid, block, 0, s>>>(c, S, B, cnew, cold, rebuild);
  }
  if (ev) (void)hipEventRecord(ev[4], s);
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

hipError_t launch_set_segments(const Ctx& c, const State& S, const Contacts& cn, hipStream_t s) {
  if (c.n > 0) k_set_segments<<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, S, cn);
  return hipGetLastError();
}

hipError_t launch_selftest(int64_t n, const double* in, const double* in2, double* out,
                           hipStream_t s) {
  if (n > 0)
    k_selftest<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, in, in2, out);
  return hipGetLastError();
}

}  // namespace sdem
