/*
 * Plain FP64 CPU oracle of the TinyDEM time step (arXiv 2507.12610).
 *
 * TEST INFRASTRUCTURE ONLY: never linked into or called by the GPU solver.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no
 * fast-math), so each floating-point operation is rounded on its own.
 *
 * One step, in the order of Section 2.3 (forces from the state at the start
 * of the step, then the semi-implicit Euler update of every particle):
 *   1. contact set = { (i,j): i<j, delta_ij >= 0 } u { (i,-m): delta_im >= 0 }
 *      (Section 2.2: delta = R_i + R_j - d >= 0; Section 3.3, mesh elements
 *      labelled by non-positive indices);
 *   2. for every contact, in key order (i ascending, then j ascending):
 *      Hertz normal force with viscous damping (Eq. fn, cn), Mindlin sliding,
 *      Kelvin-Voigt rolling and twisting forces (Eq. fs, cs, fr, ft) with
 *      their spring history and Coulomb limits (Eq. Coulombs/r/t, um,
 *      um_static, fm_kinetic, um_kinetic), torques (Section 2.2), and the
 *      pairwise antisymmetry used to update j from one evaluation
 *      (Section 3.2, Eq. antisymm_normal..antisymm_sliding);
 *   3. contacts not found again lose their springs (Section 3.2);
 *   4. integration: Eq. v, x, the SPIRAL quaternion update (Eq. spiral) with
 *      the old angular velocity, then Eq. w (Section 2.3); Stokes drag per
 *      Section 2.1.
 *
 * Readings of points the paper leaves open (the same list is in the design
 * notes of the repository):
 *   R1  relative contact velocity uses  n x (r_i w_i + r_j w_j): the contact
 *       point of j lies at +r_j n from x_j, and only this sign gives
 *       f_s^ji = -f_s^ij, which Section 3.2 asserts.
 *   R2  delta = 0 is a contact (inclusive >=); all coefficients vanish there.
 *   R3  |f_m| <= mu_m |f_n| is static (equality static).
 *   R4  projection: leave u alone if |u| = 0; if u is parallel to n (the
 *       projected length is 0) u becomes 0.
 *   R5  no clamp on a tensile normal force; Coulomb uses |f_n|.
 *   R6  mesh elements: geometric radius R_m in delta; infinite radius, mass
 *       and stiffness in the constitutive laws (R* = R_i, m* = m_i,
 *       E* = E/(1-nu^2), G* = G/(2-nu)); r_i = R_i - delta/2 also for walls.
 *   R9  right-multiplication of the quaternion, no renormalisation.
 *   M1  moving meshes (extension, generalising R14; the vibrated base of the
 *       segregation example of Section 4): each element belongs to a motion
 *       group; group g turns by |Omega_g| t about the axis Omega_g through
 *       c_g and is displaced by d_g(t) = A_g (sin(2 pi f_g t + phi_g) -
 *       sin phi_g), the axis moving with it: x(t) = c_g + d_g(t) +
 *       Rot(x0 - c_g), or x0 + d_g(t) without rotation.  The material
 *       velocity at a point p is Omega_g x (p - c_g - d_g) + d_g'(t), the
 *       wall spin Omega_g.  Without a motion table one group rotates by the
 *       parameters' mesh_omega about mesh_center (R14).
 *   S1  particle spawning (Section 3.1): at the start of each step, before
 *       the contact search, up to N_spawn attempts, while n < N_max.  Attempt
 *       a (counted over the whole run, from 0) draws four numbers from
 *       Philox4x32-10 (counter (a_lo, a_hi, 0, 0), key (seed_lo, seed_hi)),
 *       u = (k + 1/2) 2^-32: the centre s_min + u (s_max - s_min) per axis
 *       and the radius R_min + u (R_max - R_min), unless a radius is carried
 *       over from a failed attempt.  The candidate fails if it would touch
 *       (delta >= 0, R2) any particle, including those spawned earlier in the
 *       same step, or any mesh element; then its radius carries over.  New
 *       particles take the next ids, velocity v0, spin w0, orientation 1.
 *   R14 rotating mesh (extension): vertices rotate rigidly about mesh_center
 *       by angle |Omega| t; the wall velocity at the contact point
 *       c = p + R_m n is Omega x (c - mesh_center) and the relative angular
 *       velocity is w_i - Omega.  Omega = 0 gives the static mesh exactly.
 */
#include "dem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ---- small vector helpers (each op rounded separately) ------------------ */
static double dot3(const double a[3], const double b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void cross3(const double a[3], const double b[3], double o[3]) {
  double t0 = a[1] * b[2] - a[2] * b[1];
  double t1 = a[2] * b[0] - a[0] * b[2];
  double t2 = a[0] * b[1] - a[1] * b[0];
  o[0] = t0;
  o[1] = t1;
  o[2] = t2;
}
static void sub3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}

/* ---- closed forms -------------------------------------------------------- */
double orc_beta(double e_n) {
  /* beta = 1/sqrt(1 + (pi/ln e_n)^2); e_n = 1 gives pi/0 = inf -> beta = 0,
   * e_n = 0 gives pi/-inf = -0 -> beta = 1 (IEEE arithmetic). */
  double r = ORC_PI / log(e_n);
  return 1.0 / sqrt(1.0 + r * r);
}

double orc_dt_default(double R_min, double rho, double E, double nu) {
  return R_min * sqrt(rho * (1.0 - nu * nu) / E);
}

static double sphere_mass(double rho, double R) { return 4.0 / 3.0 * ORC_PI * rho * R * R * R; }

int orc_validate(const orc_params* p) {
  if (!(p->rho > 0) || !(p->E > 0)) return -1;
  if (!(p->nu > -1.0 && p->nu <= 0.5)) return -1;
  if (!(p->e_n >= 0.0 && p->e_n <= 1.0)) return -1;
  if (!(p->mu_s >= 0) || !(p->mu_r >= 0) || !(p->mu_t >= 0) || !(p->eta >= 0)) return -1;
  if (!(p->dt > 0)) return -1;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(p->g[k]) || !isfinite(p->mesh_omega[k]) || !isfinite(p->mesh_center[k]))
      return -1;
  return 0;
}

/* Closest point on a triangle (Fig. 4C), by the Voronoi-region method of
 * Ericson (Real-Time Collision Detection, 2005, Sec. 5.1.5): vertex regions,
 * edge regions, then the face interior via barycentric coordinates. */
void orc_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                                const double c[3], double out[3]) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  sub3(b, a, ab);
  sub3(c, a, ac);
  sub3(p, a, ap);
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) {
    memcpy(out, a, 3 * sizeof(double));
    return;
  }
  sub3(p, b, bp);
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) {
    memcpy(out, b, 3 * sizeof(double));
    return;
  }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    double t = d1 / (d1 - d3);
    for (int k = 0; k < 3; ++k) out[k] = a[k] + t * ab[k];
    return;
  }
  sub3(p, c, cp);
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) {
    memcpy(out, c, 3 * sizeof(double));
    return;
  }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    double t = d2 / (d2 - d6);
    for (int k = 0; k < 3; ++k) out[k] = a[k] + t * ac[k];
    return;
  }
  double va = d3 * d6 - d5 * d4;
  double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    double t = e43 / (e43 + e56);
    for (int k = 0; k < 3; ++k) out[k] = b[k] + t * (c[k] - b[k]);
    return;
  }
  double den = 1.0 / ((va + vb) + vc);
  double v = vb * den, w = vc * den;
  for (int k = 0; k < 3; ++k) out[k] = (a[k] + ab[k] * v) + ac[k] * w;
}

/* Closest point on the line segment ab (Fig. 4B), Ericson Sec. 5.1.2: the
 * projection parameter of p onto ab, clamped to the segment.  A segment of
 * zero length gives a. */
void orc_closest_point_segment(const double p[3], const double a[3], const double b[3],
                               double out[3]) {
  double ab[3], ap[3];
  sub3(b, a, ab);
  sub3(p, a, ap);
  double t = dot3(ap, ab);
  if (t <= 0.0) {
    memcpy(out, a, 3 * sizeof(double));
    return;
  }
  double dd = dot3(ab, ab);
  if (t >= dd) {
    memcpy(out, b, 3 * sizeof(double));
    return;
  }
  double u = t / dd;
  for (int k = 0; k < 3; ++k) out[k] = a[k] + u * ab[k];
}

/* Closest point on the rectangle with corners a, b, c, d in cyclic order
 * (Fig. 4D), Ericson Sec. 5.1.4: p - a is expressed along the two edges
 * e1 = b - a and e2 = d - a, which are orthogonal, and each coordinate is
 * clamped to its edge on its own.  Corner c is implied (b + d - a) and not
 * read. */
void orc_closest_point_rectangle(const double p[3], const double a[3], const double b[3],
                                 const double c[3], const double d[3], double out[3]) {
  (void)c;
  double e1[3], e2[3], ap[3];
  sub3(b, a, e1);
  sub3(d, a, e2);
  sub3(p, a, ap);
  double s1 = dot3(ap, e1), l1 = dot3(e1, e1);
  double s2 = dot3(ap, e2), l2 = dot3(e2, e2);
  double c1 = s1 >= l1 ? 1.0 : (s1 > 0.0 ? s1 / l1 : 0.0);
  double c2 = s2 >= l2 ? 1.0 : (s2 > 0.0 ? s2 / l2 : 0.0);
  for (int k = 0; k < 3; ++k) out[k] = (a[k] + c1 * e1[k]) + c2 * e2[k];
}

/* Closest point on mesh element v [4][3] with nv vertices (Section 3.3,
 * Fig. 4A-D): the vertex itself, a segment, a triangle or a rectangle. */
void orc_closest_point_element(const double p[3], int32_t nv, const double v[12], double out[3]) {
  switch (nv) {
    case 1:
      memcpy(out, v, 3 * sizeof(double));
      return;
    case 2:
      orc_closest_point_segment(p, v, v + 3, out);
      return;
    case 3:
      orc_closest_point_triangle(p, v, v + 3, v + 6, out);
      return;
    default:
      orc_closest_point_rectangle(p, v, v + 3, v + 6, v + 9, out);
      return;
  }
}

void orc_quat_mul(const double a[4], const double b[4], double out[4]) {
  /* (a0 b0 - av.bv, a0 bv + b0 av + av x bv) */
  double cr[3];
  cross3(a + 1, b + 1, cr);
  double s = a[0] * b[0] - dot3(a + 1, b + 1);
  double o1 = (a[0] * b[1] + b[0] * a[1]) + cr[0];
  double o2 = (a[0] * b[2] + b[0] * a[2]) + cr[1];
  double o3 = (a[0] * b[3] + b[0] * a[3]) + cr[2];
  out[0] = s;
  out[1] = o1;
  out[2] = o2;
  out[3] = o3;
}

/* ---- friction modes (Eq. um, um_static, fm_kinetic, um_kinetic) ---------- */
/* Vector mode m in {s, r}: project the old spring onto the tangent plane and
 * restore its length (R4), evaluate f = -k u - c v, then either keep the
 * static spring and integrate it, or clip f to mu|f_n| and reset the spring
 * so that -k u - c v reproduces the clipped force.  Returns 1 if kinetic. */
static int friction_vector(const double n[3], double k, double c, double lim, double dt,
                           const double vm[3], double u[3], double f[3]) {
  double ul = norm3(u);
  if (ul > 0.0) {
    double un = dot3(u, n);
    double up[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
    double upl = norm3(up);
    if (upl > 0.0) {
      double sc = ul / upl;
      for (int a = 0; a < 3; ++a) u[a] = up[a] * sc;
    } else {
      u[0] = u[1] = u[2] = 0.0;
    }
  }
  for (int a = 0; a < 3; ++a) f[a] = -k * u[a] - c * vm[a];
  double fl = norm3(f);
  if (fl <= lim) {
    for (int a = 0; a < 3; ++a) u[a] = u[a] + dt * vm[a];
    return 0;
  }
  double sc = lim / fl;
  for (int a = 0; a < 3; ++a) f[a] = f[a] * sc;
  for (int a = 0; a < 3; ++a) u[a] = -(f[a] + c * vm[a]) / k;
  return 1;
}

/* Twisting: the same in scalar form, no projection (Section 2.3). */
static int friction_scalar(double k, double c, double lim, double dt, double vm, double* u,
                           double* f) {
  *f = -k * (*u) - c * vm;
  if (fabs(*f) <= lim) {
    *u = *u + dt * vm;
    return 0;
  }
  *f = (*f > 0.0) ? lim : -lim;
  *u = -(*f + c * vm) / k;
  return 1;
}

/* Shared tail of both contact kinds: coefficients, forces, springs, torques.
 * Inputs are the geometry (n, delta, ri, rj; rj < 0 marks a wall), effective
 * radius/mass/moduli, the relative velocity v of the contact points, the
 * relative angular velocity om and the rolling lever reff. */
static void contact_forces(const orc_params* p, const double n[3], double delta, double Rs,
                           double ms, double Es, double Gs, const double v[3], const double om[3],
                           double reff, const double us_in[3], const double ur_in[3],
                           double ut_in, orc_contact* o) {
  double beta = orc_beta(p->e_n);
  double a = sqrt(Rs * delta);
  double kn = 4.0 / 3.0 * Es * a;
  double ks = 8.0 * Gs * a;
  double cn = sqrt(5.0 * ms * kn) * beta;
  double cs = sqrt(ms * ks / 6.0) * beta;
  double kr = kn, cr = cn, kt = ks, ct = cs; /* Section 2.2 heuristic */
  o->kn = kn;
  o->ks = ks;
  o->cn = cn;
  o->cs = cs;

  double vnn = dot3(v, n);
  for (int k = 0; k < 3; ++k) {
    o->vn[k] = vnn * n[k];
    o->vs[k] = v[k] - o->vn[k];
  }
  double oxn[3];
  cross3(om, n, oxn);
  for (int k = 0; k < 3; ++k) o->vr[k] = reff * oxn[k];
  o->vt = Rs * dot3(om, n);

  /* f_n = -k_n u_n - c_n v_n with u_n = -delta n */
  for (int k = 0; k < 3; ++k) o->fn[k] = kn * delta * n[k] - cn * o->vn[k];
  double lim_base = norm3(o->fn);

  double us[3] = {us_in[0], us_in[1], us_in[2]};
  double ur[3] = {ur_in[0], ur_in[1], ur_in[2]};
  double ut = ut_in;
  o->kinetic[0] = friction_vector(n, ks, cs, p->mu_s * lim_base, p->dt, o->vs, us, o->fs);
  o->kinetic[1] = friction_vector(n, kr, cr, p->mu_r * lim_base, p->dt, o->vr, ur, o->fr);
  o->kinetic[2] = friction_scalar(kt, ct, p->mu_t * lim_base, p->dt, o->vt, &ut, &o->ft);
  memcpy(o->us, us, sizeof us);
  memcpy(o->ur, ur, sizeof ur);
  o->ut = ut;

  /* torques: tau_s = r_i f_s x n, tau_r = R* n x f_r, tau_t = f_t R* n */
  double fsxn[3], nxfr[3];
  cross3(o->fs, n, fsxn);
  cross3(n, o->fr, nxfr);
  for (int k = 0; k < 3; ++k) {
    double ts = o->ri * fsxn[k];
    double tr = Rs * nxfr[k];
    double tt = o->ft * Rs * n[k];
    o->fi[k] = o->fn[k] + o->fs[k];
    o->ti[k] = (ts + tr) + tt;
    o->fj[k] = -o->fi[k];
    /* Eq. antisymm_sliding: tau_s^ji = r_j f_s x n; rolling, twisting flip */
    o->tj[k] = (o->rj * fsxn[k] - tr) - tt;
  }
}

int orc_eval_pp(const orc_params* p, const double xi[3], const double vi[3], const double wi[3],
                double Ri, const double xj[3], const double vj[3], const double wj[3], double Rj,
                const double us_in[3], const double ur_in[3], double ut_in, orc_contact* o) {
  double dv[3];
  sub3(xi, xj, dv);
  double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
  double delta = (Ri + Rj) - d;
  if (!(delta >= 0.0)) return 0;
  memset(o, 0, sizeof *o);
  o->d = d;
  o->delta = delta;
  for (int k = 0; k < 3; ++k) o->n[k] = dv[k] / d;
  o->ri = Ri - delta / 2.0;
  o->rj = Rj - delta / 2.0;
  double mi = sphere_mass(p->rho, Ri), mj = sphere_mass(p->rho, Rj);
  double Rs = 1.0 / (1.0 / Ri + 1.0 / Rj);
  double ms = 1.0 / (1.0 / mi + 1.0 / mj);
  double Es = p->E / (2.0 * (1.0 - p->nu * p->nu));
  double Gs = p->E / (4.0 * (2.0 - p->nu) * (1.0 + p->nu));
  /* R1: v = v_i - v_j + n x (r_i w_i + r_j w_j) */
  double rot[3], nxr[3], v[3], om[3];
  for (int k = 0; k < 3; ++k) rot[k] = o->ri * wi[k] + o->rj * wj[k];
  cross3(o->n, rot, nxr);
  for (int k = 0; k < 3; ++k) {
    v[k] = (vi[k] - vj[k]) + nxr[k];
    om[k] = wi[k] - wj[k];
  }
  double reff = 1.0 / (1.0 / o->ri + 1.0 / o->rj);
  contact_forces(p, o->n, delta, Rs, ms, Es, Gs, v, om, reff, us_in, ur_in, ut_in, o);
  return 1;
}

int orc_eval_pw(const orc_params* p, const double xi[3], const double vi[3], const double wi[3],
                double Ri, const double cp[3], double Rm, const double vwall[3],
                const double wwall[3], const double us_in[3], const double ur_in[3], double ut_in,
                orc_contact* o) {
  double dv[3];
  sub3(xi, cp, dv);
  double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
  double delta = (Ri + Rm) - d;
  if (!(delta >= 0.0)) return 0;
  memset(o, 0, sizeof *o);
  o->d = d;
  o->delta = delta;
  for (int k = 0; k < 3; ++k) o->n[k] = dv[k] / d;
  o->ri = Ri - delta / 2.0;
  o->rj = INFINITY;
  double mi = sphere_mass(p->rho, Ri);
  double Es = p->E / (1.0 - p->nu * p->nu);
  double Gs = p->E / (2.0 * (1.0 + p->nu) * (2.0 - p->nu));
  double rot[3], nxr[3], v[3], om[3];
  for (int k = 0; k < 3; ++k) rot[k] = o->ri * wi[k];
  cross3(o->n, rot, nxr);
  for (int k = 0; k < 3; ++k) {
    v[k] = (vi[k] - vwall[k]) + nxr[k];
    om[k] = wi[k] - wwall[k];
  }
  /* (1/r_i + 1/inf)^-1 = r_i */
  contact_forces(p, o->n, delta, Ri, mi, Es, Gs, v, om, o->ri, us_in, ur_in, ut_in, o);
  /* a wall takes no reaction */
  memset(o->fj, 0, sizeof o->fj);
  memset(o->tj, 0, sizeof o->tj);
  return 1;
}

/* ---- counter-based random numbers ---------------------------------------- */
/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011): each round multiplies words 0 and
 * 2 by fixed odd constants, crosses the high and low halves with the other
 * two words and the key, and bumps the key by the two Weyl constants. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
    uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
    c0 = h1 ^ c1 ^ k0;
    c1 = l1;
    c2 = h0 ^ c3 ^ k1;
    c3 = l0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* the uniform in (0, 1) of one 32-bit output: (k + 1/2) 2^-32, exact */
static double unit_open(uint32_t k) { return ((double)k + 0.5) * (1.0 / 4294967296.0); }

/* ---- simulation state ---------------------------------------------------- */
typedef struct {
  int32_t ki, kj;
  double us[3], ur[3], ut;
  double f[3], ti[3], tj[3];
} contact_rec;

struct orc_sim {
  orc_params p;
  int64_t n;
  double *x, *v, *w, *q, *R, *m, *I;
  double *F, *T, *Fs, *Ts;
  int64_t ntri;          /* mesh elements */
  int32_t* nv;           /* vertices per element, 1..4 */
  double *tri0, *tri;    /* vertices [ntri][4][3] at t = 0 and now */
  double* rmesh;         /* element radii R_m */
  int32_t* grp;          /* motion group of each element */
  int32_t ngroups;       /* 0: one group from the parameters (R14) */
  orc_motion* motion;
  double t, t0;  /* t = t0 + nstep * dt */
  /* spawning (Section 3.1) */
  int64_t cap;        /* allocated particles */
  int32_t spawn_on;
  orc_spawn sp;
  uint64_t attempts;  /* spawn attempts made so far */
  double carried;     /* radius carried over from a failed attempt, or 0 */
  int64_t nstep;
  int32_t search_mode;
  double cell_factor;
  contact_rec* hist; /* springs of the previous step, key order */
  int64_t nhist, caphist;
  /* linked cells */
  int64_t* head;
  int64_t* next;
  int64_t ncell, nxyz[3];
  double lo[3], h;
};

static void* xmalloc(size_t b) {
  void* p = malloc(b ? b : 1);
  if (!p) abort();
  return p;
}

orc_sim* orc_create(const orc_params* p, int64_t n, const double* x, const double* v,
                    const double* w, const double* q, const double* R) {
  if (orc_validate(p) != 0 || n < 0) return NULL;
  for (int64_t i = 0; i < n; ++i)
    if (!(R[i] > 0)) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof *s);
  s->p = *p;
  s->n = n;
  size_t v3 = (size_t)n * 3 * sizeof(double);
  s->x = xmalloc(v3);
  s->v = xmalloc(v3);
  s->w = xmalloc(v3);
  s->q = xmalloc((size_t)n * 4 * sizeof(double));
  s->R = xmalloc((size_t)n * sizeof(double));
  s->m = xmalloc((size_t)n * sizeof(double));
  s->I = xmalloc((size_t)n * sizeof(double));
  s->F = calloc((size_t)n * 3 + 1, sizeof(double));
  s->T = calloc((size_t)n * 3 + 1, sizeof(double));
  s->Fs = calloc((size_t)n + 1, sizeof(double));
  s->Ts = calloc((size_t)n + 1, sizeof(double));
  memcpy(s->x, x, v3);
  memcpy(s->v, v, v3);
  memcpy(s->w, w, v3);
  memcpy(s->q, q, (size_t)n * 4 * sizeof(double));
  memcpy(s->R, R, (size_t)n * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    s->m[i] = sphere_mass(p->rho, R[i]);       /* m = 4/3 pi rho R^3 */
    s->I[i] = 2.0 / 5.0 * s->m[i] * R[i] * R[i]; /* I = 2/5 m R^2     */
  }
  s->search_mode = (n <= 2048) ? 0 : 1;
  s->cell_factor = 1.0;
  s->cap = n;
  return s;
}

/* room for at least `need` particles in every per-particle array */
static void ensure_cap(orc_sim* s, int64_t need) {
  if (need <= s->cap) return;
  int64_t c = 2 * s->cap + 64;
  if (c < need) c = need;
  size_t d = sizeof(double);
  s->x = realloc(s->x, (size_t)c * 3 * d);
  s->v = realloc(s->v, (size_t)c * 3 * d);
  s->w = realloc(s->w, (size_t)c * 3 * d);
  s->q = realloc(s->q, (size_t)c * 4 * d);
  s->R = realloc(s->R, (size_t)c * d);
  s->m = realloc(s->m, (size_t)c * d);
  s->I = realloc(s->I, (size_t)c * d);
  s->F = realloc(s->F, ((size_t)c * 3 + 1) * d);
  s->T = realloc(s->T, ((size_t)c * 3 + 1) * d);
  s->Fs = realloc(s->Fs, ((size_t)c + 1) * d);
  s->Ts = realloc(s->Ts, ((size_t)c + 1) * d);
  if (!s->x || !s->v || !s->w || !s->q || !s->R || !s->m || !s->I || !s->F || !s->T || !s->Fs ||
      !s->Ts)
    abort();
  s->cap = c;
}

int orc_set_spawn(orc_sim* s, const orc_spawn* p) {
  if (!p) {
    s->spawn_on = 0;
    return 0;
  }
  for (int k = 0; k < 3; ++k)
    if (!isfinite(p->smin[k]) || !isfinite(p->smax[k]) || !(p->smax[k] >= p->smin[k]) ||
        !isfinite(p->v0[k]) || !isfinite(p->w0[k]))
      return -1;
  if (!(p->Rmin > 0) || !(p->Rmax >= p->Rmin) || !isfinite(p->Rmax)) return -1;
  if (p->n_spawn < 0 || p->n_max < 0) return -1;
  s->sp = *p;
  s->spawn_on = 1;
  s->attempts = 0;
  s->carried = 0.0;
  return 0;
}

void orc_set_spawn_status(orc_sim* s, uint64_t attempts, double carried) {
  s->attempts = attempts;
  s->carried = carried;
}

void orc_spawn_status(const orc_sim* s, uint64_t* attempts, double* carried) {
  if (attempts) *attempts = s->attempts;
  if (carried) *carried = s->carried;
}

/* would a sphere of radius r at c touch (delta >= 0) a particle or a mesh
 * element? */
static int spawn_blocked(const orc_sim* s, const double c[3], double r) {
  for (int64_t i = 0; i < s->n; ++i) {
    double dv[3];
    sub3(s->x + 3 * i, c, dv);
    double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
    if ((s->R[i] + r) - d >= 0.0) return 1;
  }
  for (int64_t m = 0; m < s->ntri; ++m) {
    double cp[3], dv[3];
    orc_closest_point_element(c, s->nv[m], s->tri + 12 * m, cp);
    sub3(c, cp, dv);
    double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
    if ((r + s->rmesh[m]) - d >= 0.0) return 1;
  }
  return 0;
}

/* the spawn attempts of one step (reading S1) */
static void spawn_step(orc_sim* s) {
  if (!s->spawn_on) return;
  const orc_spawn* p = &s->sp;
  const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
  for (int64_t k = 0; k < p->n_spawn && s->n < p->n_max; ++k) {
    uint64_t a = s->attempts++;
    uint32_t ctr[4] = {(uint32_t)a, (uint32_t)(a >> 32), 0u, 0u}, o[4];
    orc_philox4x32_10(ctr, key, o);
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = p->smin[d] + unit_open(o[d]) * (p->smax[d] - p->smin[d]);
    double r = s->carried > 0.0 ? s->carried : p->Rmin + unit_open(o[3]) * (p->Rmax - p->Rmin);
    if (spawn_blocked(s, c, r)) {
      s->carried = r;
      continue;
    }
    s->carried = 0.0;
    ensure_cap(s, s->n + 1);
    int64_t i = s->n++;
    for (int d = 0; d < 3; ++d) {
      s->x[3 * i + d] = c[d];
      s->v[3 * i + d] = p->v0[d];
      s->w[3 * i + d] = p->w0[d];
    }
    s->q[4 * i] = 1.0;
    s->q[4 * i + 1] = 0.0;
    s->q[4 * i + 2] = 0.0;
    s->q[4 * i + 3] = 0.0;
    s->R[i] = r;
    s->m[i] = sphere_mass(s->p.rho, r);
    s->I[i] = 2.0 / 5.0 * s->m[i] * r * r;
  }
}

void orc_free(orc_sim* s) {
  if (!s) return;
  free(s->x);
  free(s->v);
  free(s->w);
  free(s->q);
  free(s->R);
  free(s->m);
  free(s->I);
  free(s->F);
  free(s->T);
  free(s->Fs);
  free(s->Ts);
  free(s->tri0);
  free(s->tri);
  free(s->rmesh);
  free(s->nv);
  free(s->grp);
  free(s->motion);
  free(s->hist);
  free(s->head);
  free(s->next);
  free(s);
}

static void update_mesh(orc_sim* s);

/* A rectangle's corners must have a right angle at corner 0 and corner 2 at
 * corner 1 + corner 3 - corner 0, each to 1e-6 relative to the edges. */
static int is_rectangle(const double* v) {
  double e1[3], e2[3], g[3];
  sub3(v + 3, v, e1);
  sub3(v + 9, v, e2);
  for (int k = 0; k < 3; ++k) g[k] = v[6 + k] - ((v[3 + k] + v[9 + k]) - v[k]);
  double l1 = norm3(e1), l2 = norm3(e2);
  if (fabs(dot3(e1, e2)) > 1e-6 * l1 * l2) return 0;
  return norm3(g) <= 1e-6 * (l1 + l2);
}

int orc_set_mesh_elements(orc_sim* s, int64_t nel, const int32_t* nv, const double* verts,
                          const double* rmesh) {
  if (nel < 0) return -1;
  for (int64_t m = 0; m < nel; ++m) {
    if (nv[m] < 1 || nv[m] > 4) return -1;
    for (int k = 0; k < 3 * nv[m]; ++k)
      if (!isfinite(verts[12 * m + k])) return -1;
    if (rmesh && !(rmesh[m] >= 0 && isfinite(rmesh[m]))) return -1;
    if (nv[m] == 4 && !is_rectangle(verts + 12 * m)) return -1;
  }
  free(s->tri0);
  free(s->tri);
  free(s->rmesh);
  free(s->nv);
  free(s->grp);
  s->ntri = nel;
  s->grp = calloc((size_t)nel + 1, sizeof(int32_t));
  s->tri0 = xmalloc((size_t)nel * 12 * sizeof(double));
  s->tri = xmalloc((size_t)nel * 12 * sizeof(double));
  s->rmesh = xmalloc((size_t)nel * sizeof(double));
  s->nv = xmalloc((size_t)nel * sizeof(int32_t));
  for (int64_t m = 0; m < nel; ++m) {
    s->nv[m] = nv[m];
    /* slots past the element's own vertices repeat its last vertex */
    for (int k = 0; k < 12; ++k) {
      int slot = k / 3 < nv[m] ? k / 3 : nv[m] - 1;
      s->tri0[12 * m + k] = verts[12 * m + 3 * slot + k % 3];
    }
    s->rmesh[m] = rmesh ? rmesh[m] : 0.0;
  }
  update_mesh(s);
  return 0;
}

int orc_set_mesh(orc_sim* s, int64_t ntri, const double* tri, const double* rmesh) {
  if (ntri < 0) return -1;
  int32_t* nv = xmalloc((size_t)ntri * sizeof(int32_t));
  double* v = xmalloc((size_t)ntri * 12 * sizeof(double));
  for (int64_t m = 0; m < ntri; ++m) {
    nv[m] = 3;
    memcpy(v + 12 * m, tri + 9 * m, 9 * sizeof(double));
    memcpy(v + 12 * m + 9, tri + 9 * m + 6, 3 * sizeof(double));
  }
  int rc = orc_set_mesh_elements(s, ntri, nv, v, rmesh);
  free(nv);
  free(v);
  return rc;
}

static int key_less(int32_t ai, int32_t aj, int32_t bi, int32_t bj) {
  return ai < bi || (ai == bi && aj < bj);
}

static int cmp_rec(const void* a, const void* b) {
  const contact_rec* x = (const contact_rec*)a;
  const contact_rec* y = (const contact_rec*)b;
  if (key_less(x->ki, x->kj, y->ki, y->kj)) return -1;
  if (key_less(y->ki, y->kj, x->ki, x->kj)) return 1;
  return 0;
}

int orc_set_history(orc_sim* s, int64_t nc, const int32_t* ki, const int32_t* kj,
                    const double* us, const double* ur, const double* ut) {
  free(s->hist);
  s->hist = (contact_rec*)calloc((size_t)nc + 1, sizeof(contact_rec));
  s->caphist = nc + 1;
  s->nhist = nc;
  for (int64_t c = 0; c < nc; ++c) {
    s->hist[c].ki = ki[c];
    s->hist[c].kj = kj[c];
    for (int k = 0; k < 3; ++k) {
      s->hist[c].us[k] = us[3 * c + k];
      s->hist[c].ur[k] = ur[3 * c + k];
    }
    s->hist[c].ut = ut[c];
  }
  qsort(s->hist, (size_t)nc, sizeof(contact_rec), cmp_rec);
  return 0;
}

void orc_set_time(orc_sim* s, double t) {
  s->t = t;
  s->t0 = t;
  s->nstep = 0;
  update_mesh(s);
}
double orc_get_time(const orc_sim* s) { return s->t; }

void orc_set_search(orc_sim* s, int32_t mode, double cell_factor) {
  s->search_mode = mode;
  s->cell_factor = cell_factor >= 1.0 ? cell_factor : 1.0;
}

/* The motion of group g at time t (M1): axis direction and angle, and the
 * displacement and its velocity. */
typedef struct {
  double om[3], ctr[3];
  double wl, kx[3], co, si;  /* |Omega|, axis, cos and sin of the angle */
  double d[3], vt[3];        /* displacement d(t) and velocity d'(t)   */
} motion_now;

static const orc_motion* group_motion(const orc_sim* s, int32_t g, orc_motion* tmp) {
  if (s->ngroups > 0) return &s->motion[g];
  memset(tmp, 0, sizeof *tmp);
  memcpy(tmp->omega, s->p.mesh_omega, sizeof tmp->omega);
  memcpy(tmp->center, s->p.mesh_center, sizeof tmp->center);
  return tmp;
}

static void motion_at(const orc_motion* g, double t, motion_now* o) {
  memcpy(o->om, g->omega, sizeof o->om);
  memcpy(o->ctr, g->center, sizeof o->ctr);
  o->wl = norm3(g->omega);
  o->co = 1.0;
  o->si = 0.0;
  for (int k = 0; k < 3; ++k) o->kx[k] = 0.0;
  if (o->wl > 0.0) {
    for (int k = 0; k < 3; ++k) o->kx[k] = g->omega[k] / o->wl;
    double ang = o->wl * t;
    o->co = cos(ang);
    o->si = sin(ang);
  }
  double wv = 2.0 * ORC_PI * g->freq;
  double ph = wv * t + g->phase;
  double s1 = sin(ph) - sin(g->phase), c1 = wv * cos(ph);
  for (int k = 0; k < 3; ++k) {
    o->d[k] = g->amp[k] * s1;
    o->vt[k] = g->amp[k] * c1;
  }
}

static int is_moving(const orc_motion* g) {
  for (int k = 0; k < 3; ++k)
    if (g->omega[k] != 0.0 || (g->amp[k] != 0.0 && g->freq != 0.0)) return 1;
  return 0;
}

/* M1 (R14): vertices of every element at time t from those at t = 0 */
static void update_mesh(orc_sim* s) {
  for (int64_t m = 0; m < s->ntri; ++m) {
    orc_motion tmp;
    const orc_motion* g = group_motion(s, s->grp[m], &tmp);
    const double* x0 = s->tri0 + 12 * m;
    double* x = s->tri + 12 * m;
    if (!is_moving(g)) {
      memcpy(x, x0, 12 * sizeof(double));
      continue;
    }
    motion_now mn;
    motion_at(g, s->t, &mn);
    for (int v = 0; v < 4; ++v) {
      if (!(mn.wl > 0.0)) {
        for (int k = 0; k < 3; ++k) x[3 * v + k] = x0[3 * v + k] + mn.d[k];
        continue;
      }
      /* Rodrigues' formula about the axis through the moved centre */
      double r[3], kxr[3];
      sub3(x0 + 3 * v, mn.ctr, r);
      cross3(mn.kx, r, kxr);
      double kd = dot3(mn.kx, r);
      for (int k = 0; k < 3; ++k)
        x[3 * v + k] = (mn.ctr[k] + mn.d[k]) +
                       ((r[k] * mn.co + kxr[k] * mn.si) + mn.kx[k] * kd * (1.0 - mn.co));
    }
  }
}

/* material velocity and spin of element m's wall at the contact point */
static void wall_motion(const orc_sim* s, int64_t m, const double cpt[3], double vw[3],
                        double ww[3]) {
  orc_motion tmp;
  const orc_motion* g = group_motion(s, s->grp[m], &tmp);
  if (!is_moving(g)) {
    for (int k = 0; k < 3; ++k) vw[k] = ww[k] = 0.0;
    return;
  }
  motion_now mn;
  motion_at(g, s->t, &mn);
  double piv[3], r[3];
  for (int k = 0; k < 3; ++k) piv[k] = mn.ctr[k] + mn.d[k];
  sub3(cpt, piv, r);
  cross3(mn.om, r, vw);
  for (int k = 0; k < 3; ++k) vw[k] = vw[k] + mn.vt[k];
  memcpy(ww, mn.om, 3 * sizeof(double));
}

void orc_wall_velocity(const orc_sim* s, int64_t m, const double p[3], double vw[3],
                       double ww[3]) {
  wall_motion(s, m, p, vw, ww);
}

int orc_set_mesh_motion(orc_sim* s, int32_t ngroups, const orc_motion* g, const int32_t* grp) {
  if (ngroups < 1 || !g) return -1;
  for (int32_t k = 0; k < ngroups; ++k) {
    for (int a = 0; a < 3; ++a)
      if (!isfinite(g[k].omega[a]) || !isfinite(g[k].center[a]) || !isfinite(g[k].amp[a]))
        return -1;
    if (!isfinite(g[k].freq) || !isfinite(g[k].phase) || g[k].freq < 0) return -1;
  }
  for (int64_t m = 0; grp && m < s->ntri; ++m)
    if (grp[m] < 0 || grp[m] >= ngroups) return -1;
  free(s->motion);
  s->motion = xmalloc((size_t)ngroups * sizeof(orc_motion));
  memcpy(s->motion, g, (size_t)ngroups * sizeof(orc_motion));
  s->ngroups = ngroups;
  for (int64_t m = 0; m < s->ntri; ++m) s->grp[m] = grp ? grp[m] : 0;
  update_mesh(s);
  return 0;
}

/* previous-step springs of key (ki,kj), or NULL */
static const contact_rec* find_hist(const orc_sim* s, int32_t ki, int32_t kj) {
  int64_t lo = 0, hi = s->nhist;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    const contact_rec* r = &s->hist[mid];
    if (key_less(r->ki, r->kj, ki, kj))
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < s->nhist && s->hist[lo].ki == ki && s->hist[lo].kj == kj) return &s->hist[lo];
  return NULL;
}

/* Linked cells over the bounding box of the centres, edge cf*2*R_max
 * (Section 3.3); lists keep ascending particle order. */
static void build_cells(orc_sim* s) {
  int64_t n = s->n;
  double Rmax = 0.0;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i) {
    if (s->R[i] > Rmax) Rmax = s->R[i];
    for (int k = 0; k < 3; ++k) {
      if (s->x[3 * i + k] < lo[k]) lo[k] = s->x[3 * i + k];
      if (s->x[3 * i + k] > hi[k]) hi[k] = s->x[3 * i + k];
    }
  }
  /* small margin: rounding of the cell coordinate must not put two touching
   * spheres two cells apart */
  s->h = s->cell_factor * 2.0 * Rmax * (1.0 + 1e-9);
  s->ncell = 1;
  for (int k = 0; k < 3; ++k) {
    s->lo[k] = lo[k];
    s->nxyz[k] = (int64_t)floor((hi[k] - lo[k]) / s->h) + 1;
    s->ncell *= s->nxyz[k];
  }
  free(s->head);
  free(s->next);
  s->head = xmalloc((size_t)s->ncell * sizeof(int64_t));
  s->next = xmalloc((size_t)(n + 1) * sizeof(int64_t));
  for (int64_t c = 0; c < s->ncell; ++c) s->head[c] = -1;
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t c3[3];
    for (int k = 0; k < 3; ++k) {
      int64_t ci = (int64_t)floor((s->x[3 * i + k] - s->lo[k]) / s->h);
      if (ci < 0) ci = 0;
      if (ci >= s->nxyz[k]) ci = s->nxyz[k] - 1;
      c3[k] = ci;
    }
    int64_t c = (c3[2] * s->nxyz[1] + c3[1]) * s->nxyz[0] + c3[0];
    s->next[i] = s->head[c];
    s->head[c] = i;
  }
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* All particles j != i that could touch i (superset), ascending; returns count. */
static int64_t neighbours(const orc_sim* s, int64_t i, int only_greater, int64_t** buf,
                          int64_t* cap) {
  int64_t cnt = 0;
  if (s->search_mode == 0) {
    for (int64_t j = only_greater ? i + 1 : 0; j < s->n; ++j) {
      if (j == i) continue;
      if (cnt == *cap) {
        *cap = 2 * *cap + 16;
        *buf = realloc(*buf, (size_t)*cap * sizeof(int64_t));
      }
      (*buf)[cnt++] = j;
    }
    return cnt;
  }
  int64_t c3[3];
  for (int k = 0; k < 3; ++k) {
    int64_t ci = (int64_t)floor((s->x[3 * i + k] - s->lo[k]) / s->h);
    if (ci < 0) ci = 0;
    if (ci >= s->nxyz[k]) ci = s->nxyz[k] - 1;
    c3[k] = ci;
  }
  for (int64_t dz = -1; dz <= 1; ++dz)
    for (int64_t dy = -1; dy <= 1; ++dy)
      for (int64_t dx = -1; dx <= 1; ++dx) {
        int64_t cx = c3[0] + dx, cy = c3[1] + dy, cz = c3[2] + dz;
        if (cx < 0 || cy < 0 || cz < 0 || cx >= s->nxyz[0] || cy >= s->nxyz[1] ||
            cz >= s->nxyz[2])
          continue;
        for (int64_t j = s->head[(cz * s->nxyz[1] + cy) * s->nxyz[0] + cx]; j >= 0; j = s->next[j]) {
          if (j == i || (only_greater && j < i)) continue;
          if (cnt == *cap) {
            *cap = 2 * *cap + 16;
            *buf = realloc(*buf, (size_t)*cap * sizeof(int64_t));
          }
          (*buf)[cnt++] = j;
        }
      }
  qsort(*buf, (size_t)cnt, sizeof(int64_t), cmp_i64);
  return cnt;
}

/* Evaluate particle-wall contact of particle i with element m, if any. */
static int eval_wall(const orc_sim* s, int64_t i, int64_t m, const double* us, const double* ur,
                     double ut, orc_contact* o) {
  double cp[3];
  orc_closest_point_element(s->x + 3 * i, s->nv[m], s->tri + 12 * m, cp);
  /* contact test first, with no wall motion; motion needs the normal */
  double dv[3];
  sub3(s->x + 3 * i, cp, dv);
  double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
  double delta = (s->R[i] + s->rmesh[m]) - d;
  if (!(delta >= 0.0)) return 0;
  double nrm[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
  double cpt[3], vw[3], ww[3];
  for (int k = 0; k < 3; ++k) cpt[k] = cp[k] + s->rmesh[m] * nrm[k];
  wall_motion(s, m, cpt, vw, ww);
  return orc_eval_pw(&s->p, s->x + 3 * i, s->v + 3 * i, s->w + 3 * i, s->R[i], cp, s->rmesh[m],
                     vw, ww, us, ur, ut, o);
}

static const double ZERO3[3] = {0.0, 0.0, 0.0};

/* One particle's semi-implicit Euler + SPIRAL update (Eq. v, x, spiral, w). */
static void integrate_one(const orc_params* p, double m, double I, double R, const double F[3],
                          const double T[3], double x[3], double v[3], double w[3], double q[4]) {
  double c = 9.0 * p->eta / (2.0 * p->rho * R * R); /* Stokes drag, Section 2.1 */
  double gam = 10.0 / 3.0 * c;
  double a[3], al[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = (F[k] / m + p->g[k]) - c * v[k];
    al[k] = T[k] / I - gam * w[k];
  }
  for (int k = 0; k < 3; ++k) {
    v[k] = v[k] + p->dt * a[k];
    x[k] = x[k] + p->dt * v[k];
  }
  double wl = norm3(w);
  if (wl > 0.0) {
    double phi = p->dt * wl / 2.0;
    double sp = sin(phi) / wl;
    double r[4] = {cos(phi), sp * w[0], sp * w[1], sp * w[2]};
    double o[4];
    orc_quat_mul(q, r, o);
    memcpy(q, o, sizeof o);
  }
  double alen = norm3(al);
  if (alen > 0.0) {
    double th = (p->dt / 2.0) * (p->dt / 2.0) * alen;
    double st = sin(th) / alen;
    double r[4] = {cos(th), st * al[0], st * al[1], st * al[2]};
    double o[4];
    orc_quat_mul(q, r, o);
    memcpy(q, o, sizeof o);
  }
  for (int k = 0; k < 3; ++k) w[k] = w[k] + p->dt * al[k];
}

void orc_integrate(const orc_params* p, double R, const double F[3], const double T[3],
                   double x[3], double v[3], double w[3], double q[4]) {
  double m = sphere_mass(p->rho, R);
  integrate_one(p, m, 2.0 / 5.0 * m * R * R, R, F, T, x, v, w, q);
}

static void add_scaled_norm(double* acc, const double v[3]) { *acc += norm3(v); }

static int step_once(orc_sim* s) {
  spawn_step(s);
  int64_t n = s->n;
  memset(s->F, 0, (size_t)n * 3 * sizeof(double));
  memset(s->T, 0, (size_t)n * 3 * sizeof(double));
  double gl = norm3(s->p.g);
  for (int64_t i = 0; i < n; ++i) {
    s->Fs[i] = s->m[i] * gl;
    s->Ts[i] = 0.0;
  }
  if (s->search_mode == 1 && n > 0) build_cells(s);

  int64_t cap = s->nhist + 64, nc = 0;
  contact_rec* out = (contact_rec*)xmalloc((size_t)cap * sizeof(contact_rec));
  int64_t* nb = NULL;
  int64_t nbcap = 0;
  for (int64_t i = 0; i < n; ++i) {
    /* mesh contacts, key j = -m ascending */
    for (int64_t m = s->ntri - 1; m >= 0; --m) {
      const contact_rec* h = find_hist(s, (int32_t)i, (int32_t)-m);
      orc_contact o;
      if (!eval_wall(s, i, m, h ? h->us : ZERO3, h ? h->ur : ZERO3, h ? h->ut : 0.0, &o)) continue;
      if (nc == cap) {
        cap = 2 * cap + 64;
        out = realloc(out, (size_t)cap * sizeof(contact_rec));
      }
      contact_rec* r = &out[nc++];
      r->ki = (int32_t)i;
      r->kj = (int32_t)-m;
      memcpy(r->us, o.us, sizeof r->us);
      memcpy(r->ur, o.ur, sizeof r->ur);
      r->ut = o.ut;
      memcpy(r->f, o.fi, sizeof r->f);
      memcpy(r->ti, o.ti, sizeof r->ti);
      memset(r->tj, 0, sizeof r->tj);
      for (int k = 0; k < 3; ++k) {
        s->F[3 * i + k] += o.fi[k];
        s->T[3 * i + k] += o.ti[k];
      }
      add_scaled_norm(&s->Fs[i], o.fi);
      add_scaled_norm(&s->Ts[i], o.ti);
    }
    /* particle contacts j > i, ascending */
    int64_t nn = neighbours(s, i, 1, &nb, &nbcap);
    for (int64_t a = 0; a < nn; ++a) {
      int64_t j = nb[a];
      const contact_rec* h = find_hist(s, (int32_t)i, (int32_t)j);
      orc_contact o;
      if (!orc_eval_pp(&s->p, s->x + 3 * i, s->v + 3 * i, s->w + 3 * i, s->R[i], s->x + 3 * j,
                       s->v + 3 * j, s->w + 3 * j, s->R[j], h ? h->us : ZERO3, h ? h->ur : ZERO3,
                       h ? h->ut : 0.0, &o))
        continue;
      if (nc == cap) {
        cap = 2 * cap + 64;
        out = realloc(out, (size_t)cap * sizeof(contact_rec));
      }
      contact_rec* r = &out[nc++];
      r->ki = (int32_t)i;
      r->kj = (int32_t)j;
      memcpy(r->us, o.us, sizeof r->us);
      memcpy(r->ur, o.ur, sizeof r->ur);
      r->ut = o.ut;
      memcpy(r->f, o.fi, sizeof r->f);
      memcpy(r->ti, o.ti, sizeof r->ti);
      memcpy(r->tj, o.tj, sizeof r->tj);
      for (int k = 0; k < 3; ++k) {
        s->F[3 * i + k] += o.fi[k];
        s->T[3 * i + k] += o.ti[k];
        s->F[3 * j + k] += o.fj[k];
        s->T[3 * j + k] += o.tj[k];
      }
      add_scaled_norm(&s->Fs[i], o.fi);
      add_scaled_norm(&s->Ts[i], o.ti);
      add_scaled_norm(&s->Fs[j], o.fj);
      add_scaled_norm(&s->Ts[j], o.tj);
    }
  }
  free(nb);
  /* contacts not found this step are forgotten (Section 3.2) */
  free(s->hist);
  s->hist = out;
  s->nhist = nc;
  s->caphist = cap;

  for (int64_t i = 0; i < n; ++i)
    integrate_one(&s->p, s->m[i], s->I[i], s->R[i], s->F + 3 * i, s->T + 3 * i, s->x + 3 * i,
                  s->v + 3 * i, s->w + 3 * i, s->q + 4 * i);
  s->nstep += 1;
  s->t = s->t0 + (double)s->nstep * s->p.dt;
  update_mesh(s);
  return 0;
}

int orc_step(orc_sim* s, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; ++k)
    if (step_once(s) != 0) return -1;
  return 0;
}

void orc_get_state(const orc_sim* s, double* x, double* v, double* w, double* q) {
  size_t v3 = (size_t)s->n * 3 * sizeof(double);
  if (x) memcpy(x, s->x, v3);
  if (v) memcpy(v, s->v, v3);
  if (w) memcpy(w, s->w, v3);
  if (q) memcpy(q, s->q, (size_t)s->n * 4 * sizeof(double));
}

void orc_get_forces(const orc_sim* s, double* F, double* T, double* Fscale, double* Tscale) {
  size_t v3 = (size_t)s->n * 3 * sizeof(double);
  if (F) memcpy(F, s->F, v3);
  if (T) memcpy(T, s->T, v3);
  if (Fscale) memcpy(Fscale, s->Fs, (size_t)s->n * sizeof(double));
  if (Tscale) memcpy(Tscale, s->Ts, (size_t)s->n * sizeof(double));
}

int64_t orc_num_particles(const orc_sim* s) { return s->n; }

void orc_get_radii(const orc_sim* s, double* R) { memcpy(R, s->R, (size_t)s->n * sizeof(double)); }

int64_t orc_num_contacts(const orc_sim* s) { return s->nhist; }

void orc_get_contacts(const orc_sim* s, int32_t* ki, int32_t* kj, double* us, double* ur,
                      double* ut, double* f, double* ti, double* tj) {
  for (int64_t c = 0; c < s->nhist; ++c) {
    const contact_rec* r = &s->hist[c];
    if (ki) ki[c] = r->ki;
    if (kj) kj[c] = r->kj;
    for (int k = 0; k < 3; ++k) {
      if (us) us[3 * c + k] = r->us[k];
      if (ur) ur[3 * c + k] = r->ur[k];
      if (f) f[3 * c + k] = r->f[k];
      if (ti) ti[3 * c + k] = r->ti[k];
      if (tj) tj[3 * c + k] = r->tj[k];
    }
    if (ut) ut[c] = r->ut;
  }
}

void orc_get_mesh(const orc_sim* s, double* verts) {
  memcpy(verts, s->tri, (size_t)s->ntri * 12 * sizeof(double));
}

int64_t orc_contact_keys(orc_sim* s, int64_t cap, int32_t* ki, int32_t* kj) {
  if (s->search_mode == 1 && s->n > 0) build_cells(s);
  int64_t nc = 0;
  int64_t* nb = NULL;
  int64_t nbcap = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    for (int64_t m = s->ntri - 1; m >= 0; --m) {
      double cp[3], dv[3];
      orc_closest_point_element(s->x + 3 * i, s->nv[m], s->tri + 12 * m, cp);
      sub3(s->x + 3 * i, cp, dv);
      double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
      if ((s->R[i] + s->rmesh[m]) - d >= 0.0) {
        if (nc < cap) {
          ki[nc] = (int32_t)i;
          kj[nc] = (int32_t)-m;
        }
        ++nc;
      }
    }
    int64_t nn = neighbours(s, i, 1, &nb, &nbcap);
    for (int64_t a = 0; a < nn; ++a) {
      int64_t j = nb[a];
      double dv[3];
      sub3(s->x + 3 * i, s->x + 3 * j, dv);
      double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
      if ((s->R[i] + s->R[j]) - d >= 0.0) {
        if (nc < cap) {
          ki[nc] = (int32_t)i;
          kj[nc] = (int32_t)j;
        }
        ++nc;
      }
    }
  }
  free(nb);
  return nc;
}

int64_t orc_sample_keys(orc_sim* s, int64_t ns, const int64_t* idx, int64_t cap, int64_t* cnt,
                        int32_t* ki, int32_t* kj) {
  if (s->n > 0) build_cells(s);
  int32_t saved_mode = s->search_mode;
  s->search_mode = 1;
  int64_t* nb = NULL;
  int64_t nbcap = 0, total = 0;
  for (int64_t a = 0; a < ns; ++a) {
    int64_t p = idx[a];
    if (p < 0 || p >= s->n) {
      s->search_mode = saved_mode;
      free(nb);
      return -1;
    }
    int64_t c0 = total;
    int64_t nn = neighbours(s, p, 0, &nb, &nbcap);
    /* key order: pairs (j, p) with j < p, then (p, -m) for m descending,
     * then pairs (p, j) with j > p */
    for (int pass = 0; pass < 3; ++pass) {
      if (pass == 1) {
        for (int64_t m = s->ntri - 1; m >= 0; --m) {
          double cp[3], dv[3];
          orc_closest_point_element(s->x + 3 * p, s->nv[m], s->tri + 12 * m, cp);
          sub3(s->x + 3 * p, cp, dv);
          double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
          if ((s->R[p] + s->rmesh[m]) - d >= 0.0) {
            if (total < cap) {
              ki[total] = (int32_t)p;
              kj[total] = (int32_t)-m;
            }
            ++total;
          }
        }
        continue;
      }
      for (int64_t b = 0; b < nn; ++b) {
        int64_t j = nb[b];
        if ((pass == 0) != (j < p)) continue;
        int64_t i0 = j < p ? j : p, j0 = j < p ? p : j;
        double dv[3];
        sub3(s->x + 3 * i0, s->x + 3 * j0, dv);
        double d = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
        if ((s->R[i0] + s->R[j0]) - d >= 0.0) {
          if (total < cap) {
            ki[total] = (int32_t)i0;
            kj[total] = (int32_t)j0;
          }
          ++total;
        }
      }
    }
    if (cnt) cnt[a] = total - c0;
  }
  free(nb);
  s->search_mode = saved_mode;
  return total;
}

int orc_sample_step(orc_sim* s, int64_t ns, const int64_t* idx, double* F, double* T,
                    double* Fscale, double* Tscale, int64_t* ncont, double* x1, double* v1,
                    double* w1, double* q1) {
  if (s->n > 0) build_cells(s); /* sampled search always uses cells */
  int32_t saved_mode = s->search_mode;
  s->search_mode = 1;
  double gl = norm3(s->p.g);
  int64_t* nb = NULL;
  int64_t nbcap = 0;
  for (int64_t a = 0; a < ns; ++a) {
    int64_t p = idx[a];
    if (p < 0 || p >= s->n) {
      s->search_mode = saved_mode;
      free(nb);
      return -1;
    }
    double Fp[3] = {0, 0, 0}, Tp[3] = {0, 0, 0}, fsc = s->m[p] * gl, tsc = 0.0;
    int64_t cnt = 0;
    for (int64_t m = s->ntri - 1; m >= 0; --m) {
      const contact_rec* h = find_hist(s, (int32_t)p, (int32_t)-m);
      orc_contact o;
      if (!eval_wall(s, p, m, h ? h->us : ZERO3, h ? h->ur : ZERO3, h ? h->ut : 0.0, &o)) continue;
      ++cnt;
      for (int k = 0; k < 3; ++k) {
        Fp[k] += o.fi[k];
        Tp[k] += o.ti[k];
      }
      fsc += norm3(o.fi);
      tsc += norm3(o.ti);
    }
    int64_t nn = neighbours(s, p, 0, &nb, &nbcap);
    for (int64_t b = 0; b < nn; ++b) {
      int64_t qn = nb[b];
      int64_t i = p < qn ? p : qn, j = p < qn ? qn : p;
      const contact_rec* h = find_hist(s, (int32_t)i, (int32_t)j);
      orc_contact o;
      if (!orc_eval_pp(&s->p, s->x + 3 * i, s->v + 3 * i, s->w + 3 * i, s->R[i], s->x + 3 * j,
                       s->v + 3 * j, s->w + 3 * j, s->R[j], h ? h->us : ZERO3, h ? h->ur : ZERO3,
                       h ? h->ut : 0.0, &o))
        continue;
      ++cnt;
      const double* fp = (p == i) ? o.fi : o.fj;
      const double* tp = (p == i) ? o.ti : o.tj;
      for (int k = 0; k < 3; ++k) {
        Fp[k] += fp[k];
        Tp[k] += tp[k];
      }
      fsc += norm3(fp);
      tsc += norm3(tp);
    }
    for (int k = 0; k < 3; ++k) {
      if (F) F[3 * a + k] = Fp[k];
      if (T) T[3 * a + k] = Tp[k];
    }
    if (Fscale) Fscale[a] = fsc;
    if (Tscale) Tscale[a] = tsc;
    if (ncont) ncont[a] = cnt;
    double x[3], v[3], w[3], q[4];
    memcpy(x, s->x + 3 * p, sizeof x);
    memcpy(v, s->v + 3 * p, sizeof v);
    memcpy(w, s->w + 3 * p, sizeof w);
    memcpy(q, s->q + 4 * p, sizeof q);
    integrate_one(&s->p, s->m[p], s->I[p], s->R[p], Fp, Tp, x, v, w, q);
    if (x1) memcpy(x1 + 3 * a, x, sizeof x);
    if (v1) memcpy(v1 + 3 * a, v, sizeof v);
    if (w1) memcpy(w1 + 3 * a, w, sizeof w);
    if (q1) memcpy(q1 + 4 * a, q, sizeof q);
  }
  free(nb);
  s->search_mode = saved_mode;
  return 0;
}
