/*
 * sdem: the per-timestep hot path of a soft-sphere DEM solver (TinyDEM,
 * Vetter, arXiv 2507.12610) on AMD MI355X (gfx950), as a C ABI.
 *
 * One call of sdem_step advances every simulation of a context by whole time
 * steps.  A step is, in order (Section 2.3 and Section 3.3 of the paper):
 *   1. broad phase: bounding box of the particle centres, cubic cells of edge
 *      cell_factor * 2 R_max, particles sorted by cell;
 *   2. narrow phase: particle pairs with delta = R_i + R_j - d >= 0, found
 *      among the particles of the cells within R_i + R_max of x_i (or, between
 *      rebuilds, among the candidates recorded at the last rebuild), and
 *      particle-mesh element pairs with
 *      delta = R_i + R_m - |x_i - closest point| >= 0, the element being a
 *      point, segment, triangle or rectangle of radius R_m (Fig. 4A-D);
 *   3. contact forces and torques: Hertz normal force with damping (Eq. fn,
 *      cn), Mindlin sliding, rolling and twisting springs with Coulomb limits
 *      (Eq. fs..ft, Coulombs/r/t, um..um_kinetic), torques, and the pairwise
 *      antisymmetry that updates both bodies from one evaluation (Section 3.2);
 *      friction springs carried from the previous step by contact key;
 *   4. semi-implicit Euler for translation (Eq. v, x), SPIRAL for the
 *      orientation quaternion (Eq. spiral), then Eq. w; Stokes drag
 *      (Section 2.1).
 *
 * Conventions
 *  - Units are SI.  Vectors are structure-of-arrays: x[0..n) holds the x
 *    components, x[n..2n) y, x[2n..3n) z.  Quaternions q[4][n], scalar part
 *    first.  Radii R[n].
 *  - The persistent id of a particle is its index in the arrays given to
 *    sdem_init / sdem_init_batch.  Every read returns data ordered by id.
 *  - Contact keys (Section 3.2): (ki, kj) with ki < kj the two particle ids
 *    for a particle pair, or kj = -m <= 0 for mesh element m of the
 *    particle's own simulation (m counted from 0 in the order given to
 *    sdem_add_mesh or sdem_add_mesh_elements).
 *  - Pointers passed to sdem_init, sdem_read_* may be device or host memory;
 *    the library copies, it never keeps a caller pointer.  Mesh and history
 *    arrays are host memory.
 *  - Device memory: the caller supplies one workspace of
 *    sdem_workspace_bytes() bytes (any device allocation, 256-byte aligned)
 *    and a HIP stream; the library allocates no device memory.  All work is
 *    enqueued on that stream.  A context is not thread-safe.
 *  - Errors: every call returns an sdem_status; sdem_last_error() gives a
 *    thread-local message.  No exception crosses the ABI.
 */
#ifndef SDEM_H
#define SDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdem_ctx sdem_ctx;

typedef enum {
  SDEM_OK = 0,
  SDEM_EINVAL = -1,     /* argument outside its documented range            */
  SDEM_ECAPACITY = -2,  /* contacts, cells or elements exceed the capacity  */
  SDEM_ENONFINITE = -3, /* a position, velocity or spin became NaN or inf   */
  SDEM_EHIP = -4,       /* a HIP runtime call failed                        */
  SDEM_ESTATE = -5      /* call not allowed in the context's current state  */
} sdem_status;

typedef enum { SDEM_FP64 = 0, SDEM_MIXED = 1 } sdem_precision;

/* Parameters of one simulation: the material block of Table 2, gravity g,
 * the time step dt (> 0; Eq. dt gives the paper's default), and a rigid
 * rotation of that simulation's mesh (angular velocity mesh_omega about an
 * axis through mesh_center; zero for the static meshes of the paper).
 * Requirements (Table 2): rho > 0, E > 0, -1 < nu <= 0.5, 0 <= e_n <= 1,
 * mu_s, mu_r, mu_t >= 0, eta >= 0, dt > 0. */
typedef struct {
  double rho, E, nu, e_n, mu_s, mu_r, mu_t, eta;
  double g[3];
  double dt;
  double mesh_omega[3];
  double mesh_center[3];
} sdem_params;

/* Capacities and launch shape of a context.
 *  n_max         particles over all simulations
 *  contacts_max  contacts (particle pairs + particle-triangle) per step
 *  cells_max     grid cells per step over all simulations (the grid spans
 *                the bounding box of each simulation's centres)
 *  tri_max       mesh elements (of any kind) over all simulations
 *  nsims_max     simulations
 *  precision     SDEM_FP64: all arithmetic in double.  SDEM_MIXED: contact
 *                force and torque arithmetic in float, with double for
 *                positions, velocities, differences, the contact test,
 *                the spring updates, force sums and integration; between
 *                steps each contact's springs are kept as floats (rounded
 *                to nearest)
 *  block         reserved: 0 or a multiple of 64 in [64, 1024] (workgroups
 *                are 256 threads)
 *  detect_lanes  lanes that share one particle's contact search: 0 or 1 (one
 *                lane per particle)
 *  cell_factor   cell edge = cell_factor * 2 * R_max, >= 0.125; 0 selects 1.
 *                Each particle searches the cells within R_i + R_max of its
 *                centre, so the contact set does not depend on this value;
 *                below 1 it trades more cell ranges for fewer candidates
 *                (polydisperse systems)
 *  skin          >= 0, in units of R_max of each simulation.  0: the cells are
 *                rebuilt every step (Section 3.3).  s > 0: the cells and the
 *                particle order are kept between rebuilds, and every search
 *                reaches s R_max / 2 further (plus, should a particle drift
 *                farther than that from where it was binned, the excess,
 *                measured every step).  The cells are rebuilt at the end of
 *                each rebuild period and at the first step after such a
 *                drift that the host sees: at the end of an sdem_step call
 *                or of a period, and in contexts of 2^20 particles or more
 *                two steps after each step that keeps the cells and runs on
 *                its own: its flag is copied to pinned host memory (8 bytes
 *                that such a context allocates at init).  Steps that keep
 *                the cells run eight to a graph while the period has room,
 *                in such contexts only after a whole period without a drift.
 *                The period doubles after a period without such a drift,
 *                up to rebuild_every, and halves after one with, down to 4.
 *                The contact set is the same for every value; only the
 *                work per step changes
 *  rebuild_every with skin > 0: the longest rebuild period, >= 1; 0 selects
 *                64
 *  contacts_per_particle  contacts (pairs and mesh elements) one particle may
 *                have in a step, in [32, 4096]; 0 selects 64.  The step
 *                kernel's search keeps the first 16 it finds on chip, the
 *                rest in n * (contacts_per_particle - 16) integers of
 *                workspace.  A step where some particle has
 *                more fails with SDEM_ECAPACITY (state kept, context failed):
 *                re-init with a larger value to go on */
typedef struct {
  int64_t n_max, contacts_max, cells_max, tri_max;
  int32_t nsims_max, precision, block, detect_lanes;
  double cell_factor;
  double skin;
  int32_t rebuild_every;
  int32_t contacts_per_particle;
} sdem_config;

/* Bytes of device workspace a context with these capacities needs. */
size_t sdem_workspace_bytes(const sdem_config* cfg);

/* One simulation of n particles (n may be 0).  x, v, w [3][n], q [4][n],
 * R [n] (R > 0); v, w may be NULL (zero), q may be NULL (identity).
 * Returns SDEM_EINVAL on a bad parameter or radius, SDEM_ECAPACITY if n,
 * the workspace or nsims exceed the capacities. */
int sdem_init(sdem_ctx** out, const sdem_config* cfg, const sdem_params* params, int64_t n,
              const double* x, const double* v, const double* w, const double* q,
              const double* R, void* workspace, size_t ws_bytes, void* hip_stream);

/* Bytes of the device scratch behind sdem_init_static (one array per GPU). */
#define SDEM_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc): sdem_init of one simulation with the library's own
 * static device scratch of SDEM_STATIC_SCRATCH_BYTES per GPU in place of a
 * caller workspace.  It calls no hipMalloc, hipFree or other device
 * allocation.  The capacities must fit: if sdem_workspace_bytes(cfg)
 * exceeds the scratch it returns SDEM_ECAPACITY (nothing is touched).  The
 * scratch of a GPU is shared by every context made this way on it and keeps
 * the last context's contents: a new sdem_init_static on a GPU clears what
 * must start at zero and takes the scratch over, after which an earlier
 * static context of that GPU must not be used again; calls that overlap on
 * one GPU race.  The context is otherwise an ordinary one (all other calls,
 * sdem_destroy included).  The first call on a device looks up the
 * scratch's address there (the device current at the call). */
int sdem_init_static(sdem_ctx** out, const sdem_config* cfg, const sdem_params* params,
                     int64_t n, const double* x, const double* v, const double* w,
                     const double* q, const double* R, void* hip_stream);

/* nsims independent simulations in one context (one launch per phase for
 * all of them).  Simulation s owns particles [offsets[s], offsets[s+1]) of the
 * arrays (host array offsets, offsets[0] = 0) and has params[s]. */
int sdem_init_batch(sdem_ctx** out, const sdem_config* cfg, int32_t nsims,
                    const sdem_params* params, const int64_t* offsets, const double* x,
                    const double* v, const double* w, const double* q, const double* R,
                    void* workspace, size_t ws_bytes, void* hip_stream);

/* Sets the triangle mesh of simulation `sim` (replacing any earlier one):
 * tri [ntri][3][3] vertex coordinates (host), rmesh [ntri] element radii
 * R_m >= 0 (host, NULL for 0).  Allowed before the first step only.
 * Equivalent to sdem_add_mesh_elements with every nverts[m] = 3. */
int sdem_add_mesh(sdem_ctx* ctx, int32_t sim, int64_t ntri, const double* tri,
                  const double* rmesh);

/* Sets the mesh of simulation `sim` (replacing any earlier one) from
 * elements of one to four vertices (Section 3.3, Fig. 4A-E): a point, a line
 * segment, a triangle or a rectangle, each thickened by its own radius
 * R_m >= 0, so that a vertex acts as a sphere and an edge as a
 * spherocylinder of that radius.  A particle touches element m when
 * R_i + R_m - |x_i - closest point of the element| >= 0; the contact point
 * lies R_m from the closest point towards the particle.  Elements touch any
 * number of particles and a particle any number of elements (no merging
 * across shared edges).
 *   nverts [nel]      vertices of each element, 1..4 (host);
 *   verts [nel][4][3] coordinates (host); slots past nverts[m] are not read;
 *                     a rectangle gives its corners in cyclic order and must
 *                     have a right angle at corner 0 and corner 2 at
 *                     corner 1 + corner 3 - corner 0, each to 1e-6 relative
 *                     to its edge lengths (corner 2 is then not used);
 *   rmesh [nel]       radii R_m >= 0 (host, NULL for all 0).
 * Keys kj = -m as in the conventions above.  Allowed before the first step
 * only.  Returns SDEM_EINVAL for a vertex count outside 1..4, a non-finite
 * coordinate, a negative radius or corners that are not a rectangle, and
 * SDEM_ECAPACITY when the elements of all simulations exceed tri_max (or
 * their bins the tables sized from it); the mesh is left unchanged then,
 * except after a bin overflow, which fails the context. */
int sdem_add_mesh_elements(sdem_ctx* ctx, int32_t sim, int64_t nel, const int32_t* nverts,
                           const double* verts, const double* rmesh);

/* Prescribed rigid motion of groups of mesh elements (an extension; the
 * vibrated base of the segregation example of Section 4 is one).  Group g
 * turns with angular velocity omega about the axis through center and is
 * displaced by d(t) = amp (sin(2 pi freq t + phase) - sin(phase)), the axis
 * moving with it: a vertex x0 given at t = 0 is at
 * center + d(t) + Rot(|omega| t)(x0 - center), or x0 + d(t) without
 * rotation.  The wall's material velocity at a contact point p is
 * omega x (p - center - d(t)) + d'(t) and its angular velocity omega; they
 * enter the relative contact velocity (Section 2.2) like a moving body of
 * infinite mass.  t = steps * dt at the start of a step (sdem_set_clock). */
typedef struct {
  double omega[3];   /* angular velocity (rad/s)                           */
  double center[3];  /* a point of the rotation axis at t = 0               */
  double amp[3];     /* amplitude vector of the harmonic displacement       */
  double freq;       /* its frequency (Hz, >= 0)                            */
  double phase;      /* its phase (rad)                                     */
} sdem_mesh_motion;

/* Sets the motion groups of simulation `sim`'s mesh (after its mesh is set;
 * setting the mesh again puts every element back in group 0): ngroups
 * motions (1..16) and the group of each element, in the order given to the
 * mesh call (NULL: all in group 0).  Without this call group 0 turns with
 * the parameters' mesh_omega about mesh_center.  Element bins are built
 * over the whole region the elements sweep.  Returns SDEM_EINVAL for a bad
 * motion, count or group index. */
int sdem_set_mesh_motion(sdem_ctx* ctx, int32_t sim, int32_t ngroups,
                         const sdem_mesh_motion* motions, const int32_t* group_of);

/* Particle spawning (Section 3.1).  At the start of every step, before the
 * broad phase, up to n_spawn attempts are made while the particle count is
 * below n_max.  Attempt a (counted from 0 over the context's life, reset by
 * sdem_set_spawn) takes the four 32-bit words of Philox4x32-10 (Salmon et
 * al., SC 2011) for counter (a mod 2^32, a div 2^32, 0, 0) and key
 * (seed mod 2^32, seed div 2^32); with u = (word + 1/2) 2^-32 the candidate
 * centre is smin + u (smax - smin) per axis and its radius
 * R_min + u (R_max - R_min), unless a radius carried over from the previous
 * failed attempt is used instead.  The candidate fails if it would touch
 * (R_j + r - d >= 0, the contact test) any particle, including one spawned
 * earlier in the same step, or any mesh element; its radius then carries
 * over (possibly to the next step).  A new particle gets the next id
 * (ids stay dense: the count before it), velocity v0, spin w0, orientation
 * (1, 0, 0, 0) and no contacts.  Only centres are confined to the box, so a
 * flat box (smin = smax on an axis) spawns in a plane.  Steps that spawn run
 * one at a time and wait for the count of new particles. */
typedef struct {
  double smin[3], smax[3];  /* spawn box of the centres, smin <= smax       */
  double R_min, R_max;      /* radius range, 0 < R_min <= R_max             */
  double v0[3], w0[3];      /* initial velocity and angular velocity        */
  int64_t n_spawn;          /* attempts per step, 0..1024                   */
  int64_t n_max;            /* spawn while the count is below this          */
  uint64_t seed;            /* generator key                                */
} sdem_spawn_params;

/* Turns spawning on for simulation `sim` (p != NULL) or off (p == NULL).
 * Spawning needs a context of one simulation (sim = 0) and n_max <= the
 * context's n_max.  Resets the attempt counter and the carried radius.  A
 * larger R_max than any initial radius widens the cells (edge
 * cell_factor * 2 R_max) and the mesh reach from then on.  May be called
 * between steps.  Returns SDEM_EINVAL for a bad box, radius range, count or
 * context, SDEM_ECAPACITY for n_max above the context's n_max. */
int sdem_set_spawn(sdem_ctx* ctx, int32_t sim, const sdem_spawn_params* p);

/* Continues the spawn sequence at attempt `attempts` with a carried radius
 * (0 for none, else within [R_min, R_max]), e.g. to resume a run.  Spawning
 * must be on. */
int sdem_set_spawn_status(sdem_ctx* ctx, uint64_t attempts, double carried);

/* The particle count (host value, no wait), and if asked the attempts made
 * so far and the radius carried over (0 if none; these wait for the
 * stream). Any pointer may be NULL. */
int sdem_spawn_status(sdem_ctx* ctx, int64_t* n, uint64_t* attempts, double* carried);

/* Sets the step counter, and with it the clock t = steps * dt of moving
 * meshes (the rotating-mesh extension), e.g. to resume a run at its time.
 * The statistics of sdem_stats count from this value. */
int sdem_set_clock(sdem_ctx* ctx, int64_t steps);

/* Loads friction-spring history (host arrays): nc keys (ki, kj) as in the
 * conventions above, springs us[nc][3], ur[nc][3], ut[nc] in the orientation
 * of body ki.  Keys that are not in contact at the next step are dropped.
 * An SDEM_MIXED context rounds the springs to the nearest float. */
int sdem_set_history(sdem_ctx* ctx, int64_t nc, const int32_t* ki, const int32_t* kj,
                     const double* us, const double* ur, const double* ut);

/* Advances all simulations by nsteps steps.  Returns SDEM_ECAPACITY or
 * SDEM_ENONFINITE if a step failed; the steps before it stand, the failed
 * step is abandoned, the reads return the state and contacts at its start,
 * and the context accepts no further steps. */
int sdem_step(sdem_ctx* ctx, int64_t nsteps);

/* Measurement aid: like sdem_step, but launches each step's kernels directly
 * (no graph) with HIP events between its phases on the context's stream,
 * and returns the mean time per step of each phase in phase_ms[0..4], and in
 * phase_ms[5] the mean duration of the kernel of phase 3 alone, from start
 * and stop events attached to its dispatch (hipExtLaunchKernel):
 *   0 bounding box and grid (steps that rebuild the cells),
 *   1 cell sort and state reorder (and mesh motion),
 *   2 opening of a step that keeps the cells (step count, drift reach),
 *   3 the step kernel: narrow phase, contact forces and torques with the
 *     spring carry-over, per-particle sums and integration,
 *   4 (empty: the integration runs in phase 3).
 * phase_ms holds 6 doubles (caller-owned, host memory).  The rebuild
 * decisions and results are identical to sdem_step's. */
int sdem_step_profiled(sdem_ctx* ctx, int64_t nsteps, double* phase_ms);

/* Current state by persistent id: x, v, w [3][n], q [4][n], and the net
 * contact force F and torque T [3][n] of the last step.  Any pointer may be
 * NULL.  Synchronises the stream. */
int sdem_read_state(sdem_ctx* ctx, double* x, double* v, double* w, double* q, double* F,
                    double* T);

/* Radii R [n] by persistent id (device or host memory; n from
 * sdem_spawn_status, which grows with spawning). */
int sdem_read_radii(sdem_ctx* ctx, double* R);

/* Contacts of the last step in key order (ki ascending, then kj ascending,
 * signed) with their springs after that step: us, ur [cap][3], ut [cap]
 * (float values widened to double in an SDEM_MIXED context).
 * *n_out receives the number of contacts; at most cap are written.  Any
 * array may be NULL.  Synchronises the stream. */
int sdem_read_contacts(sdem_ctx* ctx, int64_t cap, int64_t* n_out, int32_t* ki, int32_t* kj,
                       double* us, double* ur, double* ut);

/* Steps completed, the sums over those steps of particle-pair and
 * particle-triangle contact counts (for contacts/s), and the number of steps
 * that rebuilt the cells (all of them when skin = 0).  Any pointer may be
 * NULL.  Synchronises the stream. */
int sdem_stats(sdem_ctx* ctx, int64_t* steps, int64_t* pp_contacts, int64_t* pw_contacts,
               int64_t* rebuilds);

/* HIP graphs the context has instantiated so far (*instantiated), and
 * whether capturing one failed (*failed = 1: steps are then enqueued one
 * kernel at a time).  Every graph a context replays is made at the start of
 * its first sdem_step call, so the count stays the same over later calls;
 * a caller timing steps can check that none was made inside its window.
 * Either pointer may be NULL. */
int sdem_graph_stats(sdem_ctx* ctx, int64_t* instantiated, int32_t* failed);

/* Releases the host-side context (the workspace stays the caller's). */
int sdem_destroy(sdem_ctx* ctx);

/* Thread-local message describing the last failure. */
const char* sdem_last_error(void);

/* Device self-test of the rounding the contact test relies on: out[k] =
 * sqrt(in[k]) and out[n+k] = in[k] / in2[k] computed on the GPU (device
 * arrays in, in2 [n], out [2n]).  Used to check that the device square root
 * and division are correctly rounded, as the host's are. */
int sdem_selftest_rounding(int64_t n, const double* in, const double* in2, double* out,
                           void* hip_stream);

/* Measurement aid, not an operation of the method: copies `bytes` from src
 * to dst (device memory, 16-byte aligned, not overlapping; bytes > 0 and a
 * multiple of 16) reps + 1 times with a plain streaming kernel on the given
 * stream, and writes the mean time of the last reps copies, timed with HIP
 * events, to *ms_per_copy (host).  2 * bytes / time is the HBM bandwidth such
 * a kernel reaches, the practical ceiling beside the published peak.
 * Synchronises the stream; SDEM_EINVAL for bad arguments. */
int sdem_copy_probe(const void* src, void* dst, int64_t bytes, int32_t reps, void* hip_stream,
                    double* ms_per_copy);

/* ---- file formats (Section 6 of the paper) ------------------------------ */

/* Reads a mesh in GeomView's Object File Format: "OFF", the vertex and face
 * counts (a third count is ignored), the vertices, then per face its vertex
 * count k (1..4: point, segment, triangle, rectangle with corners in cyclic
 * order), k vertex indices and optionally an index into radii[n_radii], the
 * list of mesh radii (0 when absent); '#' starts a comment.  Writes up to cap
 * elements as sdem_add_mesh_elements takes them (nverts [cap], verts
 * [cap][4][3], rmesh [cap]; any may be NULL) and the element count to
 * *nel_out (call with cap = 0 to size the arrays).  SDEM_EINVAL, with the
 * line, for a malformed file. */
int sdem_read_off(const char* path, int32_t n_radii, const double* radii, int64_t cap,
                  int64_t* nel_out, int32_t* nverts, double* verts, double* rmesh);

/* Writes the state by id as CSV: a header "id,x,y,z,vx,vy,vz,wx,wy,wz,q0,q1,
 * q2,q3,R" and one row per particle, every number to 17 significant digits
 * (read back exactly).  Overwrites the file. */
int sdem_write_csv(sdem_ctx* ctx, const char* path);

/* Reads such a CSV: columns by header name in any order, x, y, z and R
 * required, v and w zero and q the identity when absent; with an id column
 * the rows go to their ids (a permutation of 0..n-1), else in file order.
 * Arrays as sdem_init takes them (x, v, w [3][cap], q [4][cap], R [cap],
 * host; any may be NULL); *n_out is the row count, and nothing is written
 * when it exceeds cap. */
int sdem_read_csv(const char* path, int64_t cap, int64_t* n_out, double* x, double* v, double* w,
                  double* q, double* R);

/* Writes the contacts of the last step with their springs as CSV
 * ("ki,kj,usx,usy,usz,urx,ury,urz,ut", keys as in the conventions), and
 * reads such a file into the arrays sdem_set_history takes (*nc_out rows; up
 * to cap written).  With sdem_write_csv, sdem_set_clock and
 * sdem_set_spawn_status this resumes a run with its friction history. */
int sdem_write_contacts_csv(sdem_ctx* ctx, const char* path);
int sdem_read_contacts_csv(const char* path, int64_t cap, int64_t* nc_out, int32_t* ki,
                           int32_t* kj, double* us, double* ur, double* ut);

#ifdef __cplusplus
}
#endif
#endif
