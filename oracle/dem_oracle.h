/*
 * Plain FP64 CPU oracle of the soft-sphere DEM time step of TinyDEM
 * (Vetter, arXiv 2507.12610).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU solver is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product path never calls it.  It shares no code, header or constant
 * with the GPU library.
 *
 * Everything is serial double precision, built with -ffp-contract=off so
 * that every operation is rounded on its own.  Arrays are row-major:
 * vectors [n][3], quaternions [n][4] scalar part first, triangles [m][3][3].
 *
 * What each function follows is cited by section / equation / table of the
 * paper.  Readings of points the paper leaves open are listed at the top of
 * dem_oracle.c.
 */
#ifndef DEM_ORACLE_H
#define DEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Material, kinetic and simulation parameters (Table 2 material block,
 * gravity and time step), plus the rigid rotation of the mesh used by the
 * rotating-drum workload (the paper keeps meshes static; this extension
 * reduces exactly to it for mesh_omega = 0). */
typedef struct {
  double rho, E, nu, e_n, mu_s, mu_r, mu_t, eta;
  double g[3];
  double dt;
  double mesh_omega[3];  /* angular velocity of the whole mesh (rad/s)   */
  double mesh_center[3]; /* a point on the mesh rotation axis            */
} orc_params;

/* Result of one contact evaluation (Section 2.2 and 2.3). */
typedef struct {
  double delta, d, ri, rj;          /* overlap, centre distance, lever arms */
  double n[3];                      /* unit normal pointing from j to i     */
  double kn, ks, cn, cs;            /* stiffness and damping coefficients   */
  double fn[3], fs[3], fr[3], ft;   /* normal, sliding, rolling, twisting   */
  double vn[3], vs[3], vr[3], vt;   /* relative velocities                  */
  double fi[3], ti[3];              /* force and torque on body i           */
  double fj[3], tj[3];              /* force and torque on body j (pp only) */
  double us[3], ur[3], ut;          /* spring displacements after the step  */
  int32_t kinetic[3];               /* sliding / rolling / twisting branch  */
} orc_contact;

/* ---- closed-form helpers ------------------------------------------------ */
/* Damping factor beta(e_n) (Section 2.2, Eq. cn/cs). */
double orc_beta(double e_n);
/* Default time step, Eq. dt (Section 2.3). */
double orc_dt_default(double R_min, double rho, double E, double nu);
/* Closest point on triangle abc to p (region method, Fig. 4C). */
void orc_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                                const double c[3], double out[3]);
/* Closest point on segment ab to p (Fig. 4B). */
void orc_closest_point_segment(const double p[3], const double a[3], const double b[3],
                               double out[3]);
/* Closest point on rectangle abcd (corners in cyclic order, Fig. 4D). */
void orc_closest_point_rectangle(const double p[3], const double a[3], const double b[3],
                                 const double c[3], const double d[3], double out[3]);
/* Closest point on a mesh element of nv = 1..4 vertices v[4][3]. */
void orc_closest_point_element(const double p[3], int32_t nv, const double v[12], double out[3]);
/* Hamilton product out = a*b, quaternions scalar first (Eq. spiral). */
void orc_quat_mul(const double a[4], const double b[4], double out[4]);
/* Validates parameters per Table 2 "Requirements"; returns 0 or -1. */
int orc_validate(const orc_params* p);

/* ---- single contact evaluation ------------------------------------------ */
/* Particle-particle contact of i (lower id) with j.  Springs in: us_in[3],
 * ur_in[3], ut_in (zeros for a new contact).  Returns 1 if in contact
 * (delta >= 0) and fills *out, 0 otherwise. */
int orc_eval_pp(const orc_params* p, const double xi[3], const double vi[3], const double wi[3],
                double Ri, const double xj[3], const double vj[3], const double wj[3], double Rj,
                const double us_in[3], const double ur_in[3], double ut_in, orc_contact* out);
/* Particle-wall contact of i with a mesh element whose closest core point is
 * cp and whose radius is Rm.  vwall/wwall: velocity of the wall material at
 * the contact point and its angular velocity (zero for static meshes). */
int orc_eval_pw(const orc_params* p, const double xi[3], const double vi[3], const double wi[3],
                double Ri, const double cp[3], double Rm, const double vwall[3],
                const double wwall[3], const double us_in[3], const double ur_in[3], double ut_in,
                orc_contact* out);

/* One particle's update for given net force F and torque T: semi-implicit
 * Euler (Eq. v, x), SPIRAL with the old angular velocity (Eq. spiral), then
 * Eq. w; Stokes drag per Section 2.1. */
void orc_integrate(const orc_params* p, double R, const double F[3], const double T[3],
                   double x[3], double v[3], double w[3], double q[4]);

/* Prescribed rigid motion of a group of mesh elements (an extension): turns
 * with angular velocity omega about the axis through center, displaced by
 * amp (sin(2 pi freq t + phase) - sin(phase)). */
typedef struct {
  double omega[3], center[3], amp[3];
  double freq, phase;
} orc_motion;

/* Philox4x32-10 counter-based generator (Salmon et al., SC 2011). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Particle spawning (Section 3.1): box [smin, smax], radii U[Rmin, Rmax],
 * initial velocity v0 and spin w0, n_spawn attempts per step until n_max. */
typedef struct {
  double smin[3], smax[3];
  double Rmin, Rmax;
  double v0[3], w0[3];
  int64_t n_spawn, n_max;
  uint64_t seed;
} orc_spawn;

/* ---- whole simulations -------------------------------------------------- */
typedef struct orc_sim orc_sim;
orc_sim* orc_create(const orc_params* p, int64_t n, const double* x, const double* v,
                    const double* w, const double* q, const double* R);
void orc_free(orc_sim* s);
/* Mesh elements with nv[m] = 1..4 vertices (point, segment, triangle,
 * rectangle with corners in cyclic order), verts [nel][4][3] (slots past
 * nv[m] ignored), radii rmesh [nel] >= 0 (NULL for 0).  Returns -1 for a
 * bad count, coordinate or radius, or four corners that are not a
 * rectangle (right angle at corner 0, corner 2 = corner 1 + corner 3 -
 * corner 0, each to 1e-6 relative). */
int orc_set_mesh_elements(orc_sim* s, int64_t nel, const int32_t* nv, const double* verts,
                          const double* rmesh);
/* Motion groups of the mesh (after orc_set_mesh*): ngroups motions and the
 * group of each element (NULL: all in group 0).  Without this call the mesh
 * turns by the parameters' mesh_omega about mesh_center.  -1 for a bad
 * motion or group index. */
int orc_set_mesh_motion(orc_sim* s, int32_t ngroups, const orc_motion* g, const int32_t* grp);
/* Material velocity and spin of element m's wall at point p, now. */
void orc_wall_velocity(const orc_sim* s, int64_t m, const double p[3], double vw[3],
                       double ww[3]);
/* Triangles only: tri [ntri][3][3]. */
int orc_set_mesh(orc_sim* s, int64_t ntri, const double* tri, const double* rmesh);
int orc_set_history(orc_sim* s, int64_t nc, const int32_t* ki, const int32_t* kj,
                    const double* us, const double* ur, const double* ut);
/* Turns spawning on (p != NULL; resets the attempt count and the carried
 * radius) or off.  Returns -1 for a bad box, radius range or count. */
int orc_set_spawn(orc_sim* s, const orc_spawn* p);
/* Restarts the spawn sequence at attempt `attempts` with a carried radius
 * (0 for none), e.g. to resume from another run's state. */
void orc_set_spawn_status(orc_sim* s, uint64_t attempts, double carried);
/* Attempts made so far and the radius carried over (0 if none). */
void orc_spawn_status(const orc_sim* s, uint64_t* attempts, double* carried);
void orc_set_time(orc_sim* s, double t);
double orc_get_time(const orc_sim* s);
/* Contact search: 0 = brute force over all pairs, 1 = linked cells with
 * edge cell_factor*2*R_max (Section 3.3).  Both give the same set. */
void orc_set_search(orc_sim* s, int32_t mode, double cell_factor);
int orc_step(orc_sim* s, int64_t nsteps);
void orc_get_state(const orc_sim* s, double* x, double* v, double* w, double* q);
/* Net force/torque of the last step, and the force scale
 * sum_c |contribution| + m|g| used to normalise per-particle errors. */
void orc_get_forces(const orc_sim* s, double* F, double* T, double* Fscale, double* Tscale);
int64_t orc_num_particles(const orc_sim* s);
void orc_get_radii(const orc_sim* s, double* R);
int64_t orc_num_contacts(const orc_sim* s);
/* Contacts of the last step in key order (i ascending, then j ascending,
 * signed; j <= 0 labels mesh element -j), with their springs and the force
 * and torques of each contact. */
void orc_get_contacts(const orc_sim* s, int32_t* ki, int32_t* kj, double* us, double* ur,
                      double* ut, double* f, double* ti, double* tj);
/* Current mesh vertices [ntri][4][3] (slots past an element's own vertices
 * repeat its last vertex). */
void orc_get_mesh(const orc_sim* s, double* verts);

/* Sampled one-step check for large systems: for each listed particle, find
 * every contact it takes part in at the current state (brute force over a
 * linked-cell search), evaluate it with the stored springs, and return the
 * net force and torque plus the state one step later.  The simulation
 * itself is not advanced. */
int orc_sample_step(orc_sim* s, int64_t ns, const int64_t* idx, double* F, double* T,
                    double* Fscale, double* Tscale, int64_t* ncont, double* x1, double* v1,
                    double* w1, double* q1);

/* Contact keys of listed particles at the current state (Section 3.3
 * definition; linked-cell search for pairs, every triangle for walls): for
 * each idx[a], the keys of all contacts it takes part in, in key order,
 * written one particle after another (up to cap in total); cnt[a] receives
 * the particle's count.  Returns the total, or -1 on an index out of range. */
int64_t orc_sample_keys(orc_sim* s, int64_t ns, const int64_t* idx, int64_t cap, int64_t* cnt,
                        int32_t* ki, int32_t* kj);

/* Contact set only (Section 3.3 definition): writes up to cap keys, returns
 * the total number of contacts of the current state. */
int64_t orc_contact_keys(orc_sim* s, int64_t cap, int32_t* ki, int32_t* kj);

#ifdef __cplusplus
}
#endif
#endif
