/*
 * Seeded sphere placement for the synthetic workloads (input generation only:
 * no contact mechanics, no time stepping).  Random sequential addition: each
 * sphere, in the given order, takes uniformly random trial centres inside the
 * region until one overlaps no sphere placed before it.  A linked-cell grid of
 * edge 2*max(R) limits the overlap test to the 27 surrounding cells.
 * Sequential deposition with rolling (below) builds a settled pile by
 * geometry alone: no forces, no time.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), seeded by the caller; the
 * top 53 bits of each output give a double in [0, 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double unif(uint64_t* s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

/*
 * Places n spheres of radii R[] (already scaled by the caller) in the region
 *   lo <= centre - R and centre + R <= hi                    (shape 0, box)
 *   ... and (x-cx)^2 + (z-cz)^2 <= (Rc - R)^2, z <= zmax      (shape 1, drum)
 * with cyl = {cx, cz, Rc, zmax}.  Writes centres to x[n][3].  Returns the
 * number of spheres placed (fewer than n if some sphere used up
 * max_attempts trials; the rest are left unplaced), or -1 on bad input.
 */
int64_t pack_rsa(int64_t n, const double* R, const double* lo, const double* hi, int32_t shape,
                 const double* cyl, uint64_t seed, int64_t max_attempts, double* x) {
  if (n <= 0) return 0;
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (R[i] > rmax) rmax = R[i];
  if (!(rmax > 0)) return -1;
  double h = 2.0 * rmax;
  int64_t dim[3];
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) {
    if (!(hi[k] > lo[k])) return -1;
    dim[k] = (int64_t)floor((hi[k] - lo[k]) / h) + 1;
    ncell *= dim[k];
  }
  int64_t* head = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
  int64_t* next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!head || !next) {
    free(head);
    free(next);
    return -1;
  }
  for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
  uint64_t st = seed;
  int64_t placed = 0;
  for (int64_t i = 0; i < n; ++i) {
    double r = R[i];
    int ok = 0;
    double p[3];
    for (int64_t att = 0; att < max_attempts && !ok; ++att) {
      for (int k = 0; k < 3; ++k) p[k] = (lo[k] + r) + unif(&st) * ((hi[k] - lo[k]) - 2.0 * r);
      if (shape == 1) {
        double dx = p[0] - cyl[0], dz = p[2] - cyl[1];
        double lim = cyl[2] - r;
        if (lim <= 0 || dx * dx + dz * dz > lim * lim || p[2] > cyl[3]) continue;
      }
      int64_t c3[3];
      for (int k = 0; k < 3; ++k) {
        int64_t ci = (int64_t)floor((p[k] - lo[k]) / h);
        c3[k] = ci < 0 ? 0 : (ci >= dim[k] ? dim[k] - 1 : ci);
      }
      int clash = 0;
      for (int dz = -1; dz <= 1 && !clash; ++dz)
        for (int dy = -1; dy <= 1 && !clash; ++dy)
          for (int dx = -1; dx <= 1 && !clash; ++dx) {
            int64_t cx = c3[0] + dx, cy = c3[1] + dy, cz = c3[2] + dz;
            if (cx < 0 || cy < 0 || cz < 0 || cx >= dim[0] || cy >= dim[1] || cz >= dim[2]) continue;
            for (int64_t j = head[(cz * dim[1] + cy) * dim[0] + cx]; j >= 0; j = next[j]) {
              double ex = p[0] - x[3 * j], ey = p[1] - x[3 * j + 1], ez = p[2] - x[3 * j + 2];
              double s = r + R[j];
              if (ex * ex + ey * ey + ez * ez < s * s) {
                clash = 1;
                break;
              }
            }
          }
      if (clash) continue;
      ok = 1;
      for (int k = 0; k < 3; ++k) x[3 * i + k] = p[k];
      int64_t c = (c3[2] * dim[1] + c3[1]) * dim[0] + c3[0];
      next[i] = head[c];
      head[c] = i;
      ++placed;
    }
    if (!ok) break;
  }
  free(head);
  free(next);
  return placed;
}

/*
 * Sequential deposition with rolling (Visscher and Bolsterli, "Random packing
 * of equal and unequal spheres in two and three dimensions", Nature 239,
 * 1972), the geometric stand-in for pouring spheres into a container and
 * letting them settle: each sphere, in the given order, is dropped at a
 * uniformly random (x, y) from above the pile and falls straight down until
 * it touches a sphere or the floor z = 0; it then rolls downhill, over one
 * sphere (along the vertical great circle) or in the groove of two (along
 * the circle of centres touching both), until it touches the floor, comes
 * to rest in the groove's lowest point held by both, or touches a third
 * sphere and its three contact normals can carry its weight.  A support
 * that would have to pull is released and the rolling goes on; a sphere
 * that rolls off a single support past its equator falls again.  The domain
 * is periodic in x and y (periods Lx, Ly), so there are no side walls.
 */
typedef struct {
  double x, y, z;
} V3;

static V3 v3(double x, double y, double z) {
  V3 r = {x, y, z};
  return r;
}
static V3 vadd(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
static V3 vsub(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
static V3 vmul(V3 a, double s) { return v3(a.x * s, a.y * s, a.z * s); }
static double vdot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static V3 vcross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vlen(V3 a) { return sqrt(vdot(a, a)); }

typedef struct {
  const double* R;
  double* x;  // centres [n][3], x and y wrapped into [0, L)
  double Lx, Ly, h, hx, hy, rmax;
  int64_t nx, ny, nz;
  int64_t* head;
  int64_t* next;
  int overflow;  // some query found more spheres than its buffer holds
} Pile;

typedef struct {
  int64_t j;
  V3 c;  // the image of sphere j nearest the query point
} Cand;

static int64_t wrap_cell(int64_t i, int64_t n) { return ((i % n) + n) % n; }

// The spheres of the cells that cover the box |x - c.x|, |y - c.y| <= reach,
// zlo <= z <= zhi, each at its periodic image nearest c.  Returns the count
// (at most cap).
static int64_t gather_box(Pile* P, V3 c, double reach, double zlo, double zhi, Cand* out,
                          int64_t cap) {
  int64_t x0 = (int64_t)floor((c.x - reach) / P->hx), x1 = (int64_t)floor((c.x + reach) / P->hx);
  int64_t y0 = (int64_t)floor((c.y - reach) / P->hy), y1 = (int64_t)floor((c.y + reach) / P->hy);
  if (x1 - x0 + 1 > P->nx) x1 = x0 + P->nx - 1;
  if (y1 - y0 + 1 > P->ny) y1 = y0 + P->ny - 1;
  int64_t z0 = (int64_t)floor(zlo / P->h), z1 = (int64_t)floor(zhi / P->h);
  if (z0 < 0) z0 = 0;
  if (z1 > P->nz - 1) z1 = P->nz - 1;
  int64_t m = 0;
  for (int64_t iz = z0; iz <= z1; ++iz)
    for (int64_t iy = y0; iy <= y1; ++iy)
      for (int64_t ix = x0; ix <= x1; ++ix) {
        int64_t cell = (iz * P->ny + wrap_cell(iy, P->ny)) * P->nx + wrap_cell(ix, P->nx);
        for (int64_t j = P->head[cell]; j >= 0; j = P->next[j]) {
          if (m >= cap) {
            P->overflow = 1;
            return m;
          }
          double dx = P->x[3 * j] - c.x, dy = P->x[3 * j + 1] - c.y;
          dx -= P->Lx * nearbyint(dx / P->Lx);
          dy -= P->Ly * nearbyint(dy / P->Ly);
          out[m].j = j;
          out[m].c = v3(c.x + dx, c.y + dy, P->x[3 * j + 2]);
          ++m;
        }
      }
  return m;
}

// The same for the cube of half-width reach around c.
static int64_t gather(Pile* P, V3 c, double reach, Cand* out, int64_t cap) {
  return gather_box(P, c, reach, c.z - reach, c.z + reach, out, cap);
}

// First t in (t0, tmax] at which A sin t + B cos t rises through C (the
// moving centre comes within reach of a sphere), or -1.
static double first_entry(double A, double B, double C, double t0, double tmax) {
  double r0 = hypot(A, B);
  if (!(r0 > 0.0) || fabs(C) >= r0) return -1.0;
  double ph = atan2(A, B), dl = acos(C / r0);
  double t = ph - dl;
  const double tau = 2.0 * 3.14159265358979323846;
  while (t <= t0 - 0.5 * tau) t += tau;
  while (t > t0 + 0.5 * tau) t -= tau;
  if (t <= t0 + 1e-12 || t > tmax) return -1.0;
  return t;
}

// Coefficients of b in the basis {n[0..k)} by least squares (k = 2) or
// exactly (k = 3); returns 0 if the normals are (nearly) dependent.
static int decompose(const V3* n, int k, V3 b, double* coef) {
  if (k == 2) {
    double a11 = vdot(n[0], n[0]), a12 = vdot(n[0], n[1]), a22 = vdot(n[1], n[1]);
    double det = a11 * a22 - a12 * a12;
    if (fabs(det) < 1e-12) return 0;
    double r1 = vdot(n[0], b), r2 = vdot(n[1], b);
    coef[0] = (r1 * a22 - r2 * a12) / det;
    coef[1] = (r2 * a11 - r1 * a12) / det;
    return 1;
  }
  V3 c12 = vcross(n[1], n[2]);
  double det = vdot(n[0], c12);
  if (fabs(det) < 1e-12) return 0;
  coef[0] = vdot(b, c12) / det;
  coef[1] = vdot(n[0], vcross(b, n[2])) / det;
  coef[2] = vdot(n[0], vcross(n[1], b)) / det;
  return 1;
}

/*
 * Deposits n spheres of radii R[] in the given order on the floor z = 0 of
 * the periodic cell [0, Lx) x [0, Ly) (Lx, Ly at least 6 max(R)).  Writes
 * the centres to x[n][3] and the number of spheres whose rolling stopped at
 * the step limit (placed where they were) to *unsettled.  Returns n, or -1
 * on bad input or if a neighbour query overflowed its buffer (radii too
 * unequal for it).
 */
int64_t pack_deposit(int64_t n, const double* R, double Lx, double Ly, uint64_t seed, double* x,
                     int64_t* unsettled) {
  if (n <= 0) return 0;
  double rmax = 0.0, vol = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(R[i] > 0.0)) return -1;
    if (R[i] > rmax) rmax = R[i];
    vol += 4.18879020478639098 * R[i] * R[i] * R[i];
  }
  if (!(Lx >= 6.0 * rmax) || !(Ly >= 6.0 * rmax)) return -1;
  Pile P;
  P.R = R;
  P.x = x;
  P.overflow = 0;
  P.Lx = Lx;
  P.Ly = Ly;
  P.rmax = rmax;
  P.h = 2.0 * rmax;
  P.nx = (int64_t)floor(Lx / P.h);
  P.ny = (int64_t)floor(Ly / P.h);
  P.hx = Lx / (double)P.nx;
  P.hy = Ly / (double)P.ny;
  // room up to a packing fraction of 0.2 plus margin
  P.nz = (int64_t)ceil((vol / (0.2 * Lx * Ly) + 8.0 * rmax) / P.h) + 2;
  int64_t ncell = P.nx * P.ny * P.nz;
  P.head = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
  P.next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  const int64_t cap = 8192;
  Cand* cand = (Cand*)malloc((size_t)cap * sizeof(Cand));
  if (!P.head || !P.next || !cand) {
    free(P.head);
    free(P.next);
    free(cand);
    return -1;
  }
  for (int64_t c = 0; c < ncell; ++c) P.head[c] = -1;
  uint64_t st = seed;
  double ztop = 0.0;
  int64_t stuck = 0;
  const V3 up = v3(0.0, 0.0, 1.0);
  for (int64_t i = 0; i < n; ++i) {
    const double r = R[i];
    V3 p = v3(unif(&st) * Lx, unif(&st) * Ly, ztop + r + 2.0 * rmax);
    int done = 0, it = 0;
    for (; it < 400 && !done; ++it) {
      // the spheres p touches now (gap within a rounding-level tolerance)
      const double tol = 1e-9 * r;
      if (p.z - r <= tol) {
        p.z = r;
        done = 1;  // on the floor
        continue;
      }
      int64_t m = gather(&P, p, r + rmax + tol, cand, cap);
      Cand touch[8];
      int nt = 0;
      for (int64_t k = 0; k < m && nt < 8; ++k) {
        double dd = vlen(vsub(p, cand[k].c)) - (r + R[cand[k].j]);
        if (dd <= tol) touch[nt++] = cand[k];
      }
      // which contacts carry load while the sphere moves under gravity:
      // the set S whose reactions are compressive and whose motion leaves
      // every other contact (tried from the fewest supports up)
      V3 nrm[8];
      for (int q = 0; q < nt; ++q) {
        V3 d = vsub(p, touch[q].c);
        nrm[q] = vmul(d, 1.0 / vlen(d));
      }
      const V3 g = v3(0.0, 0.0, -1.0);
      int best[3] = {-1, -1, -1}, ns = -1;
      V3 acc = g;
      for (int size = 0; size <= 3 && ns < 0; ++size) {
        int idx[3] = {0, 1, 2};
        if (size > nt) break;
        for (;;) {
          V3 nn[3];
          double lam[3] = {0.0, 0.0, 0.0};
          int ok = 1;
          for (int q = 0; q < size; ++q) nn[q] = nrm[idx[q]];
          V3 a = g;
          if (size == 1) {
            lam[0] = -vdot(nn[0], g);
            a = vadd(g, vmul(nn[0], lam[0]));
          } else if (size >= 2) {
            // lam = -(N^T N)^-1 N^T g by the same decomposition of -g's part
            // in the span of the normals
            if (size == 2) {
              ok = decompose(nn, 2, vmul(g, -1.0), lam);
              if (ok) {
                a = vadd(g, vadd(vmul(nn[0], lam[0]), vmul(nn[1], lam[1])));
                // keep the part of gravity along the groove (a is the
                // least-squares residual, orthogonal to both normals)
              }
            } else {
              ok = decompose(nn, 3, vmul(g, -1.0), lam);
              a = v3(0.0, 0.0, 0.0);
            }
          }
          for (int q = 0; q < size && ok; ++q)
            if (lam[q] < -1e-12) ok = 0;
          for (int q = 0; q < nt && ok; ++q) {
            int in = 0;
            for (int u = 0; u < size; ++u) in |= idx[u] == q;
            if (!in && vdot(nrm[q], a) < -1e-12) ok = 0;
          }
          if (ok) {
            ns = size;
            for (int q = 0; q < size; ++q) best[q] = idx[q];
            acc = a;
            break;
          }
          // next combination of `size` of the nt contacts
          int q = size - 1;
          while (q >= 0 && idx[q] == nt - size + q) --q;
          if (q < 0) break;
          ++idx[q];
          for (int u = q + 1; u < size; ++u) idx[u] = idx[u - 1] + 1;
        }
      }
      if (ns < 0 || ns == 3 || vlen(acc) < 1e-9) {
        done = 1;  // at rest (or no consistent motion: stays where it is)
        continue;
      }
      if (ns == 0) {
        // fall straight down onto the highest sphere below, or the floor
        double bz = r;
        int64_t top = (int64_t)floor(p.z / P.h);
        if (top > P.nz - 1) top = P.nz - 1;
        for (int64_t iz = top; iz >= 0; --iz) {
          if ((double)(iz + 1) * P.h + r + rmax < bz) break;
          // this layer's cells within r + rmax (<= h) of the drop line
          const double zc0 = ((double)iz + 0.5) * P.h;
          int64_t mm = gather_box(&P, p, r + rmax, zc0, zc0, cand, cap);
          for (int64_t k = 0; k < mm; ++k) {
            int64_t j = cand[k].j;
            double dx = cand[k].c.x - p.x, dy = cand[k].c.y - p.y, s2 = r + R[j];
            double d2 = dx * dx + dy * dy;
            if (d2 >= s2 * s2) continue;
            double zc = cand[k].c.z + sqrt(s2 * s2 - d2);
            if (zc > bz && zc < p.z - tol) bz = zc;
          }
        }
        p.z = bz;
      } else if (ns == 1) {
        // roll over sphere A along the vertical great circle, downhill
        Cand ca = touch[best[0]];
        double rho = r + R[ca.j];
        V3 u = vsub(p, ca.c);
        double hl = hypot(u.x, u.y);
        V3 hd;
        if (hl > 1e-12 * rho) {
          hd = v3(u.x / hl, u.y / hl, 0.0);
        } else {
          double an = 6.283185307179586 * unif(&st);
          hd = v3(cos(an), sin(an), 0.0);
        }
        double th0 = atan2(hl, u.z), thmax = 0.5 * 3.14159265358979323846;
        int64_t mm = gather(&P, ca.c, rho + r + rmax, cand, cap);
        double tbest = thmax;
        for (int64_t k = 0; k < mm; ++k) {
          int64_t j = cand[k].j;
          if (j == ca.j) continue;
          V3 d = vsub(cand[k].c, ca.c);
          double s2 = r + R[j];
          double t = first_entry(2.0 * rho * vdot(hd, d), 2.0 * rho * d.z,
                                 rho * rho + vdot(d, d) - s2 * s2, th0, thmax);
          if (t >= 0.0 && t < tbest) tbest = t;
        }
        double cf = (r - ca.c.z) / rho;  // the floor: cos(theta) = cf
        if (cf > -1.0 && cf < 1.0) {
          double tf = acos(cf);
          if (tf > th0 + 1e-12 && tf < tbest) tbest = tf;
        }
        p = vadd(ca.c, vadd(vmul(hd, rho * sin(tbest)), vmul(up, rho * cos(tbest))));
      } else {
        // roll in the groove of A and B along the circle of centres
        // touching both, downhill
        Cand ca = touch[best[0]], cb = touch[best[1]];
        double ra = r + R[ca.j], rb = r + R[cb.j];
        V3 e = vsub(cb.c, ca.c);
        double dab = vlen(e);
        e = vmul(e, 1.0 / dab);
        double t0 = (ra * ra - rb * rb + dab * dab) / (2.0 * dab);
        double a2 = ra * ra - t0 * t0;
        if (!(a2 > 0.0)) {
          done = 1;
          continue;
        }
        double a = sqrt(a2);
        V3 c0 = vadd(ca.c, vmul(e, t0));
        V3 w1 = vsub(p, c0);
        w1 = vsub(w1, vmul(e, vdot(w1, e)));
        double wl = vlen(w1);
        if (!(wl > 0.0)) {
          done = 1;
          continue;
        }
        w1 = vmul(w1, 1.0 / wl);
        V3 tg = vcross(e, w1);  // the circle's tangent at p, turned downhill
        if (tg.z > 0.0) tg = vmul(tg, -1.0);
        V3 low = vsub(g, vmul(e, vdot(g, e)));
        double ll = vlen(low);
        if (ll < 1e-12 || -tg.z < 1e-12) {
          done = 1;  // at the groove's lowest point
          continue;
        }
        low = vmul(low, 1.0 / ll);
        double flow = atan2(vdot(tg, low), vdot(w1, low));
        if (!(flow > 1e-12)) {
          done = 1;
          continue;
        }
        int64_t mm = gather(&P, c0, a + r + rmax, cand, cap);
        double fbest = flow;
        for (int64_t k = 0; k < mm; ++k) {
          int64_t j = cand[k].j;
          if (j == ca.j || j == cb.j) continue;
          V3 d = vsub(cand[k].c, c0);
          double s2 = r + R[j];
          double f = first_entry(2.0 * a * vdot(tg, d), 2.0 * a * vdot(w1, d),
                                 a * a + vdot(d, d) - s2 * s2, 0.0, flow);
          if (f >= 0.0 && f < fbest) fbest = f;
        }
        {
          // the floor: c0.z + a (cos f w1.z + sin f tg.z) = r
          double f = first_entry(-a * tg.z, -a * w1.z, c0.z - r, 0.0, flow);
          if (f >= 0.0 && f < fbest) fbest = f;
        }
        p = vadd(c0, vadd(vmul(w1, a * cos(fbest)), vmul(tg, a * sin(fbest))));
      }
    }
    if (!done) ++stuck;
    p.x -= Lx * floor(p.x / Lx);
    p.y -= Ly * floor(p.y / Ly);
    if (p.x >= Lx) p.x = 0.0;
    if (p.y >= Ly) p.y = 0.0;
    x[3 * i] = p.x;
    x[3 * i + 1] = p.y;
    x[3 * i + 2] = p.z;
    int64_t iz = (int64_t)floor(p.z / P.h);
    if (iz > P.nz - 1) iz = P.nz - 1;
    if (iz < 0) iz = 0;
    int64_t cell = (iz * P.ny + wrap_cell((int64_t)floor(p.y / P.hy), P.ny)) * P.nx +
                   wrap_cell((int64_t)floor(p.x / P.hx), P.nx);
    P.next[i] = P.head[cell];
    P.head[cell] = i;
    if (p.z > ztop) ztop = p.z;
  }
  free(P.head);
  free(P.next);
  free(cand);
  if (unsettled) *unsettled = stuck;
  return P.overflow ? -1 : n;
}
