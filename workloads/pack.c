/*
 * Seeded sphere placement for the synthetic workloads (input generation only:
 * no contact mechanics, no time stepping).  Random sequential addition: each
 * sphere, in the given order, takes uniformly random trial centres inside the
 * region until one overlaps no sphere placed before it.  A linked-cell grid of
 * edge 2*max(R) limits the overlap test to the 27 surrounding cells.
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
