// HIP kernels of one DEM time step on gfx950 (MI355X).
//
// Step = bbox -> grid -> cell keys + arrival ranks -> scan of cell counts ->
// scatter -> stable reorder of the state into cell order -> contact counts ->
// scan -> contact records -> contact forces (+ spring carry-over) ->
// integration.  All kernels read the context's flag word first and do
// nothing once a capacity or finiteness error has been raised, so a failed
// step leaves the previous step's buffers untouched.
#include <math.h>

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

__device__ __forceinline__ void fatomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// ---------------------------------------------------------------------------
// 1. bounding box of the centres, per simulation (Section 3.3)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_bbox_part(Ctx c, State A) {
  if (c.ctr->flags) return;
  const int ch = blockIdx.x;
  const int b0 = c.chunks[3 * ch + 1], b1 = c.chunks[3 * ch + 2];
  const int n = c.n;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double xv = A.x[k * n + i];
      lo[k] = fmin(lo[k], xv);
      hi[k] = fmax(hi[k], xv);
      bad = bad || !isfinite(xv);
    }
  }
  __shared__ double red[6][kThreads / 64];
  __shared__ int any_bad;
  if (threadIdx.x == 0) any_bad = 0;
  __syncthreads();
  if (bad) any_bad = 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double a = lo[k], b = hi[k];
    for (int o = 32; o > 0; o >>= 1) {
      a = fmin(a, __shfl_xor(a, o, 64));
      b = fmax(b, __shfl_xor(b, o, 64));
    }
    if (lane == 0) {
      red[k][wv] = a;
      red[3 + k][wv] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double a = red[k][0], b = red[3 + k][0];
      for (int w = 1; w < nw; ++w) {
        a = fmin(a, red[k][w]);
        b = fmax(b, red[3 + k][w]);
      }
      c.part[6 * ch + k] = any_bad ? NAN : a;
      c.part[6 * ch + 3 + k] = b;
    }
  }
}

// One workgroup of kGridThreads: one wave per simulation reduces that
// simulation's partials and lays out its grid (cells of edge h over the
// bounding box); then the grids are placed one after the other in the global
// cell table (exclusive scan of the cell counts over simulations).
constexpr int kGridThreads = 1024;
constexpr int kMaxSims = 4096;

__device__ __forceinline__ int block_exclusive_scan_ll(long long* buf, int len, long long* total) {
  // buf in LDS; kGridThreads threads; each thread scans a contiguous run
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
  return 0;
}

__global__ __launch_bounds__(kGridThreads) void k_grid(Ctx c) {
  if (c.ctr->flags) return;
  __shared__ long long ncell[kMaxSims];
  __shared__ long long total;
  __shared__ int bad_total;
  if (threadIdx.x == 0) {
    bad_total = 0;
    // steps started so far (a failed step is counted; the host subtracts it)
    atomicAdd(&c.ctr->steps, 1ull);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = kGridThreads / 64;
  for (int s = wv; s < c.nsims; s += nw) {
    const int q0 = c.chunk0[s], q1 = c.chunk0[s + 1];
    double L[3] = {INFINITY, INFINITY, INFINITY}, H[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int q = q0 + lane; q < q1; q += 64) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double a = c.part[6 * q + k];
        bad = bad || isnan(a);
        L[k] = fmin(L[k], a);
        H[k] = fmax(H[k], c.part[6 * q + 3 + k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      for (int o = 32; o > 0; o >>= 1) {
        L[k] = fmin(L[k], __shfl_xor(L[k], o, 64));
        H[k] = fmax(H[k], __shfl_xor(H[k], o, 64));
      }
    bad = __any(bad);
    if (lane == 0) {
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
    }
  }
  __syncthreads();
  block_exclusive_scan_ll(ncell, c.nsims, &total);
  for (int s = threadIdx.x; s < c.nsims; s += kGridThreads) {
    const long long off = ncell[s];
    c.sg[s].cell_off = (int)(off < 0x7fffffffLL ? off : 0x7fffffffLL);
  }
  if (threadIdx.x == 0) {
    const long long tot = total;
    c.ctr->ncells = (int)(tot < (long long)c.cap_cells ? tot : (long long)c.cap_cells);
    if (bad_total) atomicOr(&c.ctr->flags, kFlagNonFinite);
    if (tot > (long long)c.cap_cells) {
      c.ctr->need_cells = (int)(tot < 0x7fffffffLL ? tot : 0x7fffffffLL);
      atomicOr(&c.ctr->flags, kFlagCapCells);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. cell keys and arrival ranks (counting sort, pass 1)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(double x, double lo, double inv_h, int dim) {
  const double f = floor((x - lo) * inv_h);
  int ci = f < 0.0 ? 0 : (f >= (double)dim ? dim - 1 : (int)f);
  return ci;
}

__global__ __launch_bounds__(kThreads) void k_keys(Ctx c, State A) {
  if (c.ctr->flags) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = c.n;
  if (i >= n) return;
  const SimGrid g = c.sg[c.sim_of[i]];
  const int cx = cell_coord(A.x[i], g.lo[0], g.inv_h, g.dim[0]);
  const int cy = cell_coord(A.x[n + i], g.lo[1], g.inv_h, g.dim[1]);
  const int cz = cell_coord(A.x[2 * n + i], g.lo[2], g.inv_h, g.dim[2]);
  const int key = g.cell_off + (cz * g.dim[1] + cy) * g.dim[0] + cx;
  c.key_tmp[i] = key;
  c.rank[i] = atomicAdd(&c.cell_cnt[key], 1);
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 (reduce / scan block sums / downsweep),
// length read from the device; optionally clears the input.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int scan_len(const int* len_dev, int len_host) {
  return len_dev ? *len_dev : len_host;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* in, const int* len_dev,
                                                              int len_host, int* bsum,
                                                              const Counters* ctr) {
  if (ctr->flags) return;
  const int len = scan_len(len_dev, len_host);
  const int chunk = (len + kScanBlocks - 1) / kScanBlocks;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(len, b0 + chunk);
  int s = 0;
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) s += in[i];
  s = wave_sum_i32(s);
  __shared__ int ws[kScanThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += ws[w];
    bsum[blockIdx.x] = t;
  }
}

// Single workgroup: exclusive scan of the block sums; writes the grand total
// to *total and checks it against cap (contact capacity) if cap >= 0.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int* bsum, int* total, Counters* ctr,
                                                           int cap) {
  if (ctr->flags) return;
  constexpr int per = kScanBlocks / kScanThreads;
  __shared__ long long ws[kScanThreads / 64];
  long long v[per];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = bsum[threadIdx.x * per + k];
    s += v[k];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wv] = x;
  __syncthreads();
  long long pre = 0;
  for (int w = 0; w < wv; ++w) pre += ws[w];
  long long run = pre + x - s;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    bsum[threadIdx.x * per + k] = (int)run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) {
    const long long all = run;
    const int tot = (int)(all < 0x7fffffffLL ? all : 0x7fffffffLL);
    if (total) *total = tot;
    if (cap >= 0 && all > (long long)cap) {
      ctr->need_contacts = tot;
      atomicOr(&ctr->flags, kFlagCapContacts);
    }
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(int* in, int* out, const int* len_dev,
                                                            int len_host, const int* bsum,
                                                            int clear_input, const Counters* ctr) {
  if (ctr->flags) return;
  const int len = scan_len(len_dev, len_host);
  const int chunk = (len + kScanBlocks - 1) / kScanBlocks;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(len, b0 + chunk);
  __shared__ int ws[kScanThreads / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = bsum[blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int base = b0; base < b1; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const int v = i < b1 ? in[i] : 0;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) ws[wv] = x;
    __syncthreads();
    int pre = carry;
    for (int w = 0; w < wv; ++w) pre += ws[w];
    if (i < b1) {
      out[i] = pre + x - v;
      if (clear_input) in[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {
      int t = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
      carry += t;
    }
    __syncthreads();
  }
}

// out[len] = in-sum: separate tiny kernel so that the scan stays simple.
__global__ void k_scan_end(const int* len_dev, int len_host, int* out, const int* total,
                           const Counters* ctr) {
  if (ctr->flags) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) out[scan_len(len_dev, len_host)] = *total;
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
__global__ __launch_bounds__(kThreads) void k_reorder(Ctx c, State A, State B) {
  if (c.ctr->flags) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = c.n;
  if (p >= n) return;
  const int so = c.perm[p];
  const int k = c.key_tmp[so];
  const int cs = c.cell_start[k], ce = c.cell_start[k + 1];
  int r = 0;
  for (int t = cs; t < ce; ++t) r += (c.perm[t] < so) ? 1 : 0;
  const int d = cs + r;
#pragma unroll
  for (int k3 = 0; k3 < 3; ++k3) {
    B.x[k3 * n + d] = A.x[k3 * n + so];
    B.v[k3 * n + d] = A.v[k3 * n + so];
    B.w[k3 * n + d] = A.w[k3 * n + so];
  }
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4) B.q[k4 * n + d] = A.q[k4 * n + so];
  B.R[d] = A.R[so];
  B.pid[d] = A.pid[so];
  B.key[d] = k;
  B.src[d] = so;
}

// ---------------------------------------------------------------------------
// 4. mesh: rigid rotation (extension for rotating drums) and plane data
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mesh(Ctx c, int all) {
#pragma clang fp contract(off)
  if (c.ctr->flags) return;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= c.ntri) return;
  const SimParams& P = c.sp[c.tri_sim[m]];
  double* t = c.tri + 9 * m;
  const double* t0 = c.tri_ref + 9 * m;
  if (all) {  // set-up: vertices at t = 0
    for (int k = 0; k < 9; ++k) t[k] = t0[k];
  } else if (P.rotating) {
    // rigid rotation by |om| t about the axis om/|om| through ctr, with t the
    // time at the start of this step (steps already counted the current one)
    const double wl = sqrt((P.om[0] * P.om[0] + P.om[1] * P.om[1]) + P.om[2] * P.om[2]);
    const double kx = P.om[0] / wl, ky = P.om[1] / wl, kz = P.om[2] / wl;
    const double ang = wl * ((double)(c.ctr->steps - 1ull) * P.dt);
    const double co = cos(ang), si = sin(ang);
    for (int v = 0; v < 3; ++v) {
      const double rx = t0[3 * v] - P.ctr[0], ry = t0[3 * v + 1] - P.ctr[1],
                   rz = t0[3 * v + 2] - P.ctr[2];
      const double cx = ky * rz - kz * ry, cy = kz * rx - kx * rz, cz = kx * ry - ky * rx;
      const double kd = (kx * rx + ky * ry) + kz * rz;
      t[3 * v] = P.ctr[0] + ((rx * co + cx * si) + kx * kd * (1.0 - co));
      t[3 * v + 1] = P.ctr[1] + ((ry * co + cy * si) + ky * kd * (1.0 - co));
      t[3 * v + 2] = P.ctr[2] + ((rz * co + cz * si) + kz * kd * (1.0 - co));
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
  } else {  // degenerate element: no plane filter
    c.tri_pl[4 * m] = 0.0;
    c.tri_pl[4 * m + 1] = 0.0;
    c.tri_pl[4 * m + 2] = 0.0;
    c.tri_pl[4 * m + 3] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 5. narrow phase (Section 3.3): triangles of the particle's simulation, then
//    particle pairs in the upper half of the 27-cell neighbourhood.  With
//    cells in (z, y, x) row order the three cells cx-1..cx+1 of a row are one
//    contiguous slot range, so the half shell is five ranges: the rest of the
//    own row (slots after this one), the row at (y+1, z), and the three rows
//    at z+1.  Each pair is found once, by its lower slot (the owner).
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(kThreads) void k_detect(Ctx c, State S, Contacts cn) {
  if (c.ctr->flags) return;
  const int n = c.n;
  const int s = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int npp = 0, npw = 0;
  if (s < n) {
    const int sim = c.sim_of[s];
    const SimGrid g = c.sg[sim];
    const int tri0 = c.sp[sim].tri0, ntri = c.sp[sim].ntri;
    const double xs = S.x[s], ys = S.x[n + s], zs = S.x[2 * n + s], Rs = S.R[s];
    const int my = S.pid[s];
    int w = WRITE ? cn.off[s] : 0;
    // ---- triangles
    for (int m = tri0; m < tri0 + ntri; ++m) {
      const double* pl = c.tri_pl + 4 * m;
      const double reach = Rs + c.rmesh[m];
      const double pd = (pl[0] * xs + pl[1] * ys + pl[2] * zs) - pl[3];
      if (fabs(pd) > reach * (1.0 + 1e-9) + 1e-300) continue;
      const double p[3] = {xs, ys, zs};
      double cp[3];
      closest_on_triangle(p, c.tri + 9 * m, cp);
      double dx, dy, dz, d;
      const double delta = pair_gap(xs, ys, zs, Rs, cp[0], cp[1], cp[2], c.rmesh[m], &dx, &dy, &dz, &d);
      if (delta >= 0.0) {
        if (WRITE) {
          cn.a[w] = s;
          cn.b[w] = -1 - m;
          cn.ki[w] = my;
          cn.kj[w] = -(m - tri0);
          ++w;
        }
        ++npw;
      }
    }
    // ---- particles
    const int loc = S.key[s] - g.cell_off;
    const int nx = g.dim[0], ny = g.dim[1], nz = g.dim[2];
    const int cx = loc % nx, cyz = loc / nx, cy = cyz % ny, cz = cyz / ny;
    const int xlo = cx > 0 ? cx - 1 : 0, xhi = cx + 1 < nx ? cx + 1 : nx - 1;
    for (int r = 0; r < 5; ++r) {
      int yy, zz;
      if (r == 0) {
        yy = cy;
        zz = cz;
      } else if (r == 1) {
        yy = cy + 1;
        zz = cz;
      } else {
        yy = cy + (r - 3);
        zz = cz + 1;
      }
      if (yy < 0 || yy >= ny || zz >= nz) continue;
      const int row = g.cell_off + (zz * ny + yy) * nx;
      const int t0 = (r == 0) ? s + 1 : c.cell_start[row + xlo];
      const int t1 = c.cell_start[row + xhi + 1];
      for (int t = t0; t < t1; ++t) {
        const double xt = S.x[t], yt = S.x[n + t], zt = S.x[2 * n + t], Rt = S.R[t];
        const double ex = xs - xt, ey = ys - yt, ez = zs - zt;
        const double sr = Rs + Rt;
        // cheap conservative reject before the exactly rounded test
        if ((ex * ex + ey * ey) + ez * ez > sr * sr * (1.0 + 1e-9)) continue;
        double dx, dy, dz, d;
        const double delta = pair_gap(xs, ys, zs, Rs, xt, yt, zt, Rt, &dx, &dy, &dz, &d);
        if (delta >= 0.0) {
          if (WRITE) {
            const int ot = S.pid[t];
            cn.a[w] = s;
            cn.b[w] = t;
            cn.ki[w] = my < ot ? my : ot;
            cn.kj[w] = my < ot ? ot : my;
            ++w;
          }
          ++npp;
        }
      }
    }
    if (!WRITE) {
      cn.cnt[s] = npp + npw;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c.F[k * n + s] = 0.0;
        c.T[k * n + s] = 0.0;
      }
    }
  }
  if (!WRITE) {
    // contact counts for the statistics: one 64-bit atomic per wave
    const int a = wave_sum_i32(npp), b = wave_sum_i32(npw);
    if ((threadIdx.x & 63) == 0 && (a | b)) {
      atomicAdd(&c.ctr->pp_sum, (unsigned long long)a);
      atomicAdd(&c.ctr->pw_sum, (unsigned long long)b);
    }
  }
}

// ---------------------------------------------------------------------------
// 6. contact forces and torques (Section 2.2, 2.3, 3.2)
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
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = -((double)f[a] + (double)cdmp * (double)vm[a]) / (double)k;
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

// Finds the springs of key (ki, kj) among the previous step's contacts of the
// previous owner slot po; returns true and the springs if present.
__device__ __forceinline__ bool find_old(const Contacts& co, int po, int ki, int kj, double us[3],
                                         double ur[3], double* ut, int cap) {
  const int b0 = co.off[po], b1 = b0 + co.cnt[po];
  for (int e = b0; e < b1; ++e) {
    if (co.ki[e] == ki && co.kj[e] == kj) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        us[a] = co.us[a * cap + e];
        ur[a] = co.ur[a * cap + e];
      }
      *ut = co.ut[e];
      return true;
    }
  }
  return false;
}

template <typename RT>
__global__ __launch_bounds__(kThreads) void k_force(Ctx c, State S, Contacts cur, Contacts old) {
  if (c.ctr->flags) return;
  const int n = c.n;
  const int cap = c.cap_contacts;
  const int C = c.ctr->ncontacts;
  // contiguous chunk of contacts per workgroup, chunks grouped per XCD
  const int nb = gridDim.x;
  const int lb = xcd_remap(blockIdx.x, nb);
  const int per = ((C + nb - 1) / nb + (int)blockDim.x - 1) / (int)blockDim.x * (int)blockDim.x;
  const int e0 = lb * per;
  const int e1 = min(C, e0 + per);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int a = cur.a[e], b = cur.b[e];
    const int ki = cur.ki[e], kj = cur.kj[e];
    const int sim = c.sim_of[a];
    const SimParams& P = c.sp[sim];
    const bool wall = b < 0;
    // canonical orientation: body I carries the lower id (a for walls)
    int I = a, J = b;
    if (!wall && S.pid[a] > S.pid[b]) {
      I = b;
      J = a;
    }
    const double xi = S.x[I], yi = S.x[n + I], zi = S.x[2 * n + I], Ri = S.R[I];
    double xj, yj, zj, Rj;
    double vjx = 0.0, vjy = 0.0, vjz = 0.0, wjx = 0.0, wjy = 0.0, wjz = 0.0;
    if (!wall) {
      xj = S.x[J];
      yj = S.x[n + J];
      zj = S.x[2 * n + J];
      Rj = S.R[J];
      vjx = S.v[J];
      vjy = S.v[n + J];
      vjz = S.v[2 * n + J];
      wjx = S.w[J];
      wjy = S.w[n + J];
      wjz = S.w[2 * n + J];
    } else {
      const int m = -1 - b;
      const double p[3] = {xi, yi, zi};
      double cp[3];
      closest_on_triangle(p, c.tri + 9 * m, cp);
      xj = cp[0];
      yj = cp[1];
      zj = cp[2];
      Rj = c.rmesh[m];
    }
    double dx, dy, dz, d;
    const double delta = pair_gap(xi, yi, zi, Ri, xj, yj, zj, Rj, &dx, &dy, &dz, &d);
    const double invd = 1.0 / d;
    const RT nrm[3] = {(RT)(dx * invd), (RT)(dy * invd), (RT)(dz * invd)};
    const double ri = Ri - 0.5 * delta;
    const double mi = sphere_mass(P.rho, Ri);
    double rj, Rs, ms, Es, Gs, reff;
    double vrel[3], om[3];
    const double vix = S.v[I], viy = S.v[n + I], viz = S.v[2 * n + I];
    const double wix = S.w[I], wiy = S.w[n + I], wiz = S.w[2 * n + I];
    if (!wall) {
      rj = Rj - 0.5 * delta;
      const double mj = sphere_mass(P.rho, Rj);
      Rs = 1.0 / (1.0 / Ri + 1.0 / Rj);
      ms = 1.0 / (1.0 / mi + 1.0 / mj);
      Es = P.Es_pp;
      Gs = P.Gs_pp;
      reff = 1.0 / (1.0 / ri + 1.0 / rj);
      // v = v_i - v_j + n x (r_i w_i + r_j w_j)
      const double rx = ri * wix + rj * wjx, ry = ri * wiy + rj * wjy, rz = ri * wiz + rj * wjz;
      const double n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
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
      Es = P.Es_pw;
      Gs = P.Gs_pw;
      reff = ri;
      double vw[3] = {0.0, 0.0, 0.0};
      if (P.rotating) {  // wall material velocity at the contact point c = p + R_m n
        const double px = xj + Rj * (double)nrm[0] - P.ctr[0];
        const double py = yj + Rj * (double)nrm[1] - P.ctr[1];
        const double pz = zj + Rj * (double)nrm[2] - P.ctr[2];
        vw[0] = P.om[1] * pz - P.om[2] * py;
        vw[1] = P.om[2] * px - P.om[0] * pz;
        vw[2] = P.om[0] * py - P.om[1] * px;
      }
      const double n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
      const double rx = ri * wix, ry = ri * wiy, rz = ri * wiz;
      vrel[0] = (vix - vw[0]) + (n1 * rz - n2 * ry);
      vrel[1] = (viy - vw[1]) + (n2 * rx - n0 * rz);
      vrel[2] = (viz - vw[2]) + (n0 * ry - n1 * rx);
      om[0] = wix - P.om[0];
      om[1] = wiy - P.om[1];
      om[2] = wiz - P.om[2];
    }
    // coefficients (Eq. ks, cn, cs; k_r = k_n, c_r = c_n, k_t = k_s, c_t = c_s)
    const RT ac = (RT)sqrt(Rs * delta);
    const RT kn = (RT)(4.0 / 3.0) * (RT)Es * ac;
    const RT ks = (RT)8.0 * (RT)Gs * ac;
    const RT cn = sqrt((RT)5.0 * (RT)ms * kn) * (RT)P.beta;
    const RT cs = sqrt((RT)ms * ks / (RT)6.0) * (RT)P.beta;
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
    // springs of the previous step (zero for a new contact)
    double us[3] = {0.0, 0.0, 0.0}, ur[3] = {0.0, 0.0, 0.0}, ut = 0.0;
    {
      const int pa = S.src[a];
      const int po = wall ? pa : min(pa, S.src[b]);
      find_old(old, po, ki, kj, us, ur, &ut, cap);
    }
    RT fs[3], fr[3], ft;
    friction_vec<RT>(nrm, ks, cs, (RT)P.mu_s * fnl, P.dt, vs, us, fs);
    friction_vec<RT>(nrm, kn, cn, (RT)P.mu_r * fnl, P.dt, vr, ur, fr);
    friction_scalar<RT>(ks, cs, (RT)P.mu_t * fnl, P.dt, vt, &ut, &ft);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cur.us[k * cap + e] = us[k];
      cur.ur[k * cap + e] = ur[k];
    }
    cur.ut[e] = ut;
    // torques: tau_s = r_i f_s x n, tau_r = R* n x f_r, tau_t = f_t R* n
    const RT fsxn[3] = {fs[1] * nrm[2] - fs[2] * nrm[1], fs[2] * nrm[0] - fs[0] * nrm[2],
                        fs[0] * nrm[1] - fs[1] * nrm[0]};
    const RT rs = (RT)Rs;
    const RT tr[3] = {rs * (nrm[1] * fr[2] - nrm[2] * fr[1]), rs * (nrm[2] * fr[0] - nrm[0] * fr[2]),
                      rs * (nrm[0] * fr[1] - nrm[1] * fr[0])};
    const RT ftr = ft * rs;
    const RT rif = (RT)ri, rjf = (RT)rj;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double f = (double)fn[k] + (double)fs[k];
      const double ttr = (double)tr[k] + (double)(ftr * nrm[k]);
      const double ti = (double)(rif * fsxn[k]) + ttr;
      fatomic_add(&c.F[k * n + I], f);
      fatomic_add(&c.T[k * n + I], ti);
      if (!wall) {
        const double tj = (double)(rjf * fsxn[k]) - ttr;
        fatomic_add(&c.F[k * n + J], -f);
        fatomic_add(&c.T[k * n + J], tj);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 7. integration: semi-implicit Euler (Eq. v, x), SPIRAL (Eq. spiral) with
//    the old angular velocity, then Eq. w; Stokes drag (Section 2.1)
// ---------------------------------------------------------------------------
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

__global__ __launch_bounds__(kThreads) void k_integrate(Ctx c, State S) {
  if (c.ctr->flags) return;
  const int n = c.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const SimParams& P = c.sp[c.sim_of[i]];
    const double R = S.R[i];
    const double m = sphere_mass(P.rho, R);
    const double I = 0.4 * m * R * R;
    const double cd = 9.0 * P.eta / (2.0 * P.rho * R * R);
    const double gd = (10.0 / 3.0) * cd;
    const double dt = P.dt;
    double v[3], x[3], w[3], al[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[k] = S.v[k * n + i];
      x[k] = S.x[k * n + i];
      w[k] = S.w[k * n + i];
      const double a = (c.F[k * n + i] / m + P.g[k]) - cd * v[k];
      al[k] = c.T[k * n + i] / I - gd * w[k];
      v[k] = v[k] + dt * a;
      x[k] = x[k] + dt * v[k];
    }
    double q[4] = {S.q[i], S.q[n + i], S.q[2 * n + i], S.q[3 * n + i]};
    const double wl = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
    if (wl > 0.0) {
      const double phi = 0.5 * dt * wl;
      double sp, cp;
      sincos(phi, &sp, &cp);
      sp /= wl;
      const double r[4] = {cp, sp * w[0], sp * w[1], sp * w[2]};
      double o[4];
      qmul(q, r, o);
      q[0] = o[0]; q[1] = o[1]; q[2] = o[2]; q[3] = o[3];
    }
    const double alen = sqrt((al[0] * al[0] + al[1] * al[1]) + al[2] * al[2]);
    if (alen > 0.0) {
      const double th = (0.5 * dt) * (0.5 * dt) * alen;
      double st, ct;
      sincos(th, &st, &ct);
      st /= alen;
      const double r[4] = {ct, st * al[0], st * al[1], st * al[2]};
      double o[4];
      qmul(q, r, o);
      q[0] = o[0]; q[1] = o[1]; q[2] = o[2]; q[3] = o[3];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      w[k] = w[k] + dt * al[k];
      ok = ok && isfinite(x[k]) && isfinite(v[k]) && isfinite(w[k]);
      S.v[k * n + i] = v[k];
      S.x[k * n + i] = x[k];
      S.w[k * n + i] = w[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) S.q[k * n + i] = q[k];
    if (!ok) atomicOr(&c.ctr->flags, kFlagNonFinite);
  }
}

// ---------------------------------------------------------------------------
// reads: scatter a state buffer back to persistent-id order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_scatter_state(Ctx c, State S, double* x, double* v,
                                                            double* w, double* q, double* F,
                                                            double* T) {
  const int n = c.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int id = S.pid[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (x) x[k * n + id] = S.x[k * n + i];
    if (v) v[k * n + id] = S.v[k * n + i];
    if (w) w[k * n + id] = S.w[k * n + i];
    if (F) F[k * n + id] = c.F[k * n + i];
    if (T) T[k * n + id] = c.T[k * n + i];
  }
  if (q) {
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k * n + id] = S.q[k * n + i];
  }
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

static hipError_t scan(int* in, int* out, const int* len_dev, int len_host, int* total,
                       int clear_input, Counters* ctr, int cap, int* tmp, hipStream_t s) {
  k_scan_reduce<<<kScanBlocks, kScanThreads, 0, s>>>(in, len_dev, len_host, tmp, ctr);
  k_scan_top<<<1, kScanThreads, 0, s>>>(tmp, total, ctr, cap);
  k_scan_down<<<kScanBlocks, kScanThreads, 0, s>>>(in, out, len_dev, len_host, tmp, clear_input,
                                                   ctr);
  k_scan_end<<<1, 64, 0, s>>>(len_dev, len_host, out, total, ctr);
  return hipGetLastError();
}

hipError_t launch_step(const Ctx& c, const State& A, const State& B, const Contacts& cold,
                       const Contacts& cnew, int precision, hipStream_t s, hipEvent_t* ev) {
  // ev (optional): kPhases + 1 events recorded at the phase boundaries
  const int n = c.n;
  const int nbp = blocks_for(n, kThreads);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (c.nchunks > 0) k_bbox_part<<<c.nchunks, kThreads, 0, s>>>(c, A);
  k_grid<<<1, kGridThreads, 0, s>>>(c);
  if (ev) (void)hipEventRecord(ev[1], s);
  k_keys<<<nbp, kThreads, 0, s>>>(c, A);
  // cell starts; clears the counts for the next step; total = n
  hipError_t e = scan(c.cell_cnt, c.cell_start, &c.ctr->ncells, 0, c.scan_tmp + kScanBlocks, 1,
                      c.ctr, -1, c.scan_tmp, s);
  if (e) return e;
  k_scatter<<<nbp, kThreads, 0, s>>>(c);
  k_reorder<<<nbp, kThreads, 0, s>>>(c, A, B);
  if (c.ntri > 0) k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 0);
  if (ev) (void)hipEventRecord(ev[2], s);
  k_detect<false><<<nbp, kThreads, 0, s>>>(c, B, cnew);
  e = scan(cnew.cnt, cnew.off, nullptr, n, &c.ctr->ncontacts, 0, c.ctr, c.cap_contacts,
           c.scan_tmp, s);
  if (e) return e;
  k_detect<true><<<nbp, kThreads, 0, s>>>(c, B, cnew);
  if (ev) (void)hipEventRecord(ev[3], s);
  if (precision == SDEM_MIXED)
    k_force<float><<<kForceBlocks, kThreads, 0, s>>>(c, B, cnew, cold);
  else
    k_force<double><<<kForceBlocks, kThreads, 0, s>>>(c, B, cnew, cold);
  if (ev) (void)hipEventRecord(ev[4], s);
  k_integrate<<<nbp, kThreads, 0, s>>>(c, B);
  if (ev) (void)hipEventRecord(ev[5], s);
  return hipGetLastError();
}

hipError_t launch_scatter_state(const Ctx& c, const State& S, double* x, double* v, double* w,
                                double* q, double* F, double* T, hipStream_t s) {
  if (c.n > 0)
    k_scatter_state<<<blocks_for(c.n, kThreads), kThreads, 0, s>>>(c, S, x, v, w, q, F, T);
  return hipGetLastError();
}

hipError_t launch_mesh_planes(const Ctx& c, hipStream_t s) {
  if (c.ntri > 0) k_mesh<<<blocks_for(c.ntri, kThreads), kThreads, 0, s>>>(c, 1);
  return hipGetLastError();
}

hipError_t launch_selftest(int64_t n, const double* in, const double* in2, double* out,
                           hipStream_t s) {
  if (n > 0)
    k_selftest<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, in, in2, out);
  return hipGetLastError();
}

}  // namespace sdem
