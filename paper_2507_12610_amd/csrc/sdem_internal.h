// Internal definitions of the sdem HIP library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdem.h"

namespace sdem {

constexpr int kScanBlocks = 1024;   // fixed grid of the device-wide scan
constexpr int kScanThreads = 256;
constexpr int kPart = 7;            // doubles per bounding-box partial: min xyz, max xyz,
                                    // largest drift from the binned centre
constexpr int kWave = 64;           // slots per wave; bounding-box partials are
                                    // per (wave of slots, simulation)
constexpr int kSpr = 8;             // doubles per contact spring record
constexpr int kThreads = 256;       // threads per workgroup of the particle kernels
constexpr int kHit = 16;            // contacts of one particle held in LDS by its search
constexpr int kMinHitCap = 32;      // least contacts_per_particle a config may ask for
                                    // lane (more spill to the tile's global overflow)
constexpr int kCand = 32;           // candidates one search lane records at a rebuild
constexpr int kGroupShift = 8;      // contact records are allocated per group of
constexpr int kGroup = 1 << kGroupShift;  // 256 consecutive slots: a tile of the step kernel
constexpr int kLdsRec = 2560;       // records of a tile held in LDS (the rest in global memory)
constexpr int kLdsRef = 1536;       // in-tile references held in LDS (the rest in global memory)
constexpr int kBrickBits = 3;       // cells are ordered in bricks of up to 8 x 8 x 8
constexpr int kBinScanThreads = 1024;  // one workgroup scans the triangle bins
constexpr int kSpawnMax = 1024;     // spawn attempts per step at most
constexpr int kMotionMax = 16;      // motion groups of a simulation's mesh

enum : int {
  kFlagCapContacts = 1,
  kFlagCapCells = 2,
  kFlagNonFinite = 4,
  kFlagCapPerParticle = 8,
  kFlagCapBins = 16,
};

// Per-simulation constants, derived on the host at init.
struct SimParams {
  double rho, E, nu, e_n, mu_s, mu_r, mu_t, eta;
  double g[3];
  double dt;
  double beta;                 // 1/sqrt(1 + (pi/ln e_n)^2)
  double Es_pp, Gs_pp;         // uniform material, two spheres
  double Es_pw, Gs_pw;         // sphere against a rigid wall
  double cnf_pp, csf_pp;       // beta sqrt(20/3 E*), beta sqrt(4/3 G*): damping
  double cnf_pw, csf_pw;       // coefficients per sqrt(m* a), two spheres / wall
  double h;                    // cell edge
  double rmax;                 // largest radius of the simulation
  double half_skin;            // skin * rmax / 2: allowed drift from the binned position
  int32_t moving;              // some element of the mesh moves
  int32_t tri0, ntri;          // global triangle range
  int32_t p0, np;              // particle range (fixed positions in sorted order)
  int32_t frame_bins;          // the mesh moves as one rigid body: its element bins
                               // are built once in the mesh's own frame (t = 0) and
                               // looked up with the particle mapped back to it
};

// Prescribed rigid motion of a group of mesh elements: turns with angular
// velocity omega about the axis through center, displaced by
// amp (sin(2 pi freq t + phase) - sin(phase)), the axis moving with it.
struct MeshMotion {
  double omega[3], center[3], amp[3];
  double freq, phase;
  int32_t moving;  // omega != 0, or amp != 0 with freq != 0
  int32_t pad;
};

// Per-simulation grid of the current step (computed on the device).  Cells
// are numbered brick by brick: bricks of 2^bits[a] cells along axis a
// (bits[a] = min(3, ceil(log2 dim[a]))), bricks in (z, y, x) row order,
// the cells of a brick in Morton (bit-interleaved) order, so that a run of
// consecutive slots is a compact blob of space.
struct SimGrid {
  double lo[3];
  double inv_h;
  int32_t dim[3];
  int32_t cell_off;
  int32_t bits[3];
  int32_t nb[3];  // bricks along each axis
};

// Per-simulation uniform grid of triangle bins, fixed at set-up.  Bin b lists
// every triangle whose bounding box, grown by R_max + R_m, overlaps it; the
// grid covers all such boxes (for a rotating mesh, at every angle), so a
// particle outside it touches no triangle.
struct MeshGrid {
  double lo[3];
  double inv_h;
  int32_t dim[3];
  int32_t off;  // first bin of this simulation in the bin tables
};

// Device-side counters and flags of a context.
struct Counters {
  int32_t flags;
  int32_t need_group;    // contacts a slot group needed beyond its share (diagnostic)
  int32_t pad0;
  int32_t ncells;        // cells of the step in progress (all sims)
  int32_t need_cells;    // last required cell capacity (diagnostic)
  uint32_t scan_ticket;  // last-block detection of the scan
  int32_t rebuild_next;  // a particle drifted beyond half the skin since the last rebuild
  int32_t drift_now;     // the step in progress reaches past the skin (set by k_begin)
  int32_t pad;
  unsigned long long steps;  // steps started (a failed one included)
  unsigned long long rebuilds;  // steps that rebuilt the cells
  unsigned long long drift_steps;  // steps whose searches reached past the skin
  unsigned long long spawn_attempts;  // spawn attempts made so far
  double spawn_carried;  // radius carried over from a failed attempt, 0 if none
  int32_t spawn_new;     // particles the last spawn placed
  int32_t pad3;
};

// Particle spawning (Section 3.1) of simulation `sim`: attempts per step, the
// box of the centres, the radius range, the initial velocity and spin, the
// cap on the particle count and the generator key.
struct SpawnParams {
  double smin[3], smax[3];
  double Rmin, Rmax;
  double v0[3], w0[3];
  int32_t n_spawn, sim;
  int64_t n_max;
  uint32_t key[2];
};

// What the contact law needs of a particle besides its centre and radius, in
// one 64-byte record, so that gathering a contact partner touches its centre
// (which the search has just read) and one more 64-byte sector.
struct alignas(64) Aux {
  double2 vw[3];  // velocity (vx, vy), (vz, wx), (wy, wz): velocity then spin
  int32_t pid;    // persistent id
  int32_t prev;   // slot of the particle in the previous step's order
  int32_t off;    // its first owned record in the previous step's contacts
  int32_t cnt;    // and how many it owned
};
static_assert(sizeof(Aux) == 64, "one 64-byte sector per particle");

// One buffer of per-particle state in cell-sorted order.  The centres are an
// array of their own: the search reads many neighbours' centres and nothing
// else of them.
struct State {
  double4* xr;  // [n] centre x, y, z and radius R
  Aux* a;       // [n]
  double4* q;   // [n] orientation quaternion, scalar first
};

// The slot that owns the pair of slots a != b (evaluates it first-hand and
// keeps its springs): the lower slot when the two lie in different groups of
// kGroup; within a group, the lower slot when a + b is even and the higher
// when it is odd, so that every particle owns about half of its pairs in the
// group (the step kernel's search lanes then carry balanced loads).
__host__ __device__ inline bool slot_owns(int a, int b) {
  if ((a >> kGroupShift) != (b >> kGroupShift)) return a < b;
  return ((a ^ b) & 1) ? a > b : a < b;
}

// One buffer of contacts, grouped by owner slot (owner by slot_owns; a
// particle owns its mesh contacts).  The owned records of slot group g
// (slots g*256 .. g*256+255) live in [g*gcap, g*gcap + ng[g]), each owner's
// contiguous.  a, b hold the step kernel's work list of the tile: the owned
// records, then the records of pairs with a lower slot outside the tile
// (evaluated by both tiles), at [2*g*gcap, ...) for records past the LDS.
struct Contacts {
  int32_t* cnt;  // [n] contacts per owner slot
  int32_t* off;  // [n] first contact of each owner slot
  int32_t* a;    // [2 cap] work list: slot within the tile
  int32_t* b;    // [2 cap] work list: partner slot (>= 0) or -1 - global element index
  int32_t* ref;  // [cap] in-tile references past the LDS: record of the owning partner
  int2* key;     // (lower persistent id, higher id) or (id, -local triangle index)
  double* spr;   // [cap][kSpr] sliding spring (3), rolling spring (3), twisting
                 // spring (1), in the orientation of body key.x; one pad
  int32_t* ng;   // [ngroups] owned records of each slot group
};

// Everything a step's kernels read or write.
struct Ctx {
  int32_t n, nsims, ntri, cap_contacts, cap_cells, nchunks;
  int32_t any_moving;        // some simulation's mesh moves
  int32_t rebin;             // some moving mesh needs its bins rebuilt every step
  int32_t skin_on;           // cells are kept between steps (skin > 0)
  int32_t hit_cap;           // contacts one particle may have in a step (>= kHit)
  int32_t ngroups, gcap;     // slot groups, contact records per group
  int32_t nbins, cap_bin_entries;  // triangle bins (all sims), capacity of bin_tri
  int32_t* gcnt;             // [ngroups] contact records used by each group
  unsigned long long* gstat; // [ngroups][2] pair and wall contacts of each group, summed
                             // over the steps
  SimParams* sp;      // [nsims]
  SimGrid* sg;        // [nsims]
  int32_t* sim_of;    // [n] simulation of each slot (fixed)
  int32_t* wchunk;    // [n/64] first bounding-box chunk of each wave of slots
  int32_t* chunk0;    // [nsims+1] first chunk of each simulation
  double* xtra;       // [nsims] extra reach of the step in progress (drift past the skin)
  double* part;       // [nchunks][kPart] bounding-box partials (min xyz, max xyz, drift),
                      // one per (wave, simulation) segment, simulations ascending
  int32_t* cell_cnt;  // [cap_cells] zero between steps
  int32_t* cell_start;// [cap_cells+1]
  int32_t* key_tmp;   // [n] cell key by previous slot
  int32_t* rank;      // [n] arrival rank in the cell
  int32_t* perm;      // [n] new slot -> previous slot (unstable within a cell)
  int32_t* scan_tmp;  // [kScanBlocks+1]
  int32_t* spill;     // [n][hit_cap - kHit] contacts of a particle past its kHit in LDS
  // per slot, written by the reorder at a rebuild and kept until the next:
  double4* xb;        // [n] centre when the cells were built (w unused)
  int32_t* vcnt;      // [n] candidates recorded by each particle at the last
                      // rebuild (-1: more than kCand, search the cells)
  int32_t* vlist;     // [kCand][vstride] their slots, in search order: entry k of
                      // slot s at k * vstride + s (the first entries of a wave's
                      // slots are read together)
  int64_t vstride;    // slots the candidate lists have room for
  double* F;          // [3][n] contact force of the last step, by slot
  double* T;          // [3][n] contact torque of the last step, by slot
  double* tri_ref;    // [ntri][9] element vertices at t = 0 (see closest_on_element)
  double* tri;        // [ntri][9] element vertices at the current step
  int32_t* tri_nv;    // [ntri] vertices per element, 1..4
  double* tri_pl;     // [ntri][4] unit normal and offset of the plane
  double* rmesh;      // [ntri]
  int32_t* tri_sim;   // [ntri]
  int32_t* tri_grp;   // [ntri] motion of each element: sim * kMotionMax + group
  MeshMotion* motion; // [nsims * kMotionMax]
  double* tri_mv;     // [ntri][9] wall motion now: spin, moved centre, translation
                      // velocity (zero for elements that do not move)
  double* frame;      // [nsims][12] motion now of a mesh binned in its own frame:
                      // unit axis, cos and sin of the angle, moved centre, centre
  MeshGrid* mg;       // [nsims]
  int32_t* bin_cnt;   // [nbins] zero between builds
  int32_t* bin_start; // [nbins+1]
  int32_t* bin_tri;   // [cap_bin_entries] triangles of each bin, ascending
  Counters* ctr;
  SpawnParams* spawn;       // [1]
  double4* spawn_cand;      // [kSpawnMax] candidate centre and radius fraction
  unsigned long long* spawn_thr;  // [kSpawnMax] smallest radius that would touch
                            // something, per candidate (bits of a double >= 0)
};

// Grids up to this many workgroups are resident all at once (four per CU
// on 256 CUs).
constexpr int kOneRoundBlocks = 1024;

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // The dispatcher hands workgroup b to XCD b % 8.  When the whole grid is
  // resident at once, each XCD gets one contiguous range of logical blocks,
  // so that its L2 holds one share of the slots and their neighbours (200k
  // spheres: 3 % faster steps).  Larger grids are swept by all XCDs through
  // the same region of the sorted state together (8M spheres: 2 % faster
  // than contiguous ranges), each XCD taking 8 consecutive blocks at a time
  // so that neighbouring blocks share its L2 (a further 1.5 %); the blocks
  // past the last whole round of chunks keep their places.
  if (nb > kOneRoundBlocks) {
    constexpr int kC = 8, kS = 8 * kC;
    if (b >= (nb / kS) * kS) return b;
    const int x = b & 7, idx = b >> 3;
    return ((idx / kC) * 8 + x) * kC + idx % kC;
  }
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

// ---------------------------------------------------------------------------
// Exact-rounding geometry shared by the contact search and the force kernel:
// every operation rounded on its own (no contraction), square root and
// division correctly rounded, so the contact decision is reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pair_gap(double xi, double yi, double zi, double Ri, double xj,
                                           double yj, double zj, double Rj, double* dx, double* dy,
                                           double* dz, double* d) {
#pragma clang fp contract(off)
  const double ex = xi - xj, ey = yi - yj, ez = zi - zj;
  const double dd = sqrt((ex * ex + ey * ey) + ez * ez);
  *dx = ex;
  *dy = ey;
  *dz = ez;
  *d = dd;
  return (Ri + Rj) - dd;  // delta; contact iff >= 0
}

// Closest point of triangle (a, b, c) to p by Voronoi regions (vertex, edge,
// face), after Ericson, Real-Time Collision Detection (2005), Sec. 5.1.5.
__device__ __forceinline__ void closest_on_triangle(const double p[3], const double* t,
                                                    double out[3]) {
#pragma clang fp contract(off)
  const double a0 = t[0], a1 = t[1], a2 = t[2];
  const double ab0 = t[3] - a0, ab1 = t[4] - a1, ab2 = t[5] - a2;
  const double ac0 = t[6] - a0, ac1 = t[7] - a1, ac2 = t[8] - a2;
  const double ap0 = p[0] - a0, ap1 = p[1] - a1, ap2 = p[2] - a2;
  const double d1 = (ab0 * ap0 + ab1 * ap1) + ab2 * ap2;
  const double d2 = (ac0 * ap0 + ac1 * ap1) + ac2 * ap2;
  if (d1 <= 0.0 && d2 <= 0.0) {
    out[0] = a0; out[1] = a1; out[2] = a2;
    return;
  }
  const double bp0 = p[0] - t[3], bp1 = p[1] - t[4], bp2 = p[2] - t[5];
  const double d3 = (ab0 * bp0 + ab1 * bp1) + ab2 * bp2;
  const double d4 = (ac0 * bp0 + ac1 * bp1) + ac2 * bp2;
  if (d3 >= 0.0 && d4 <= d3) {
    out[0] = t[3]; out[1] = t[4]; out[2] = t[5];
    return;
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    const double s = d1 / (d1 - d3);
    out[0] = a0 + s * ab0; out[1] = a1 + s * ab1; out[2] = a2 + s * ab2;
    return;
  }
  const double cp0 = p[0] - t[6], cp1 = p[1] - t[7], cp2 = p[2] - t[8];
  const double d5 = (ab0 * cp0 + ab1 * cp1) + ab2 * cp2;
  const double d6 = (ac0 * cp0 + ac1 * cp1) + ac2 * cp2;
  if (d6 >= 0.0 && d5 <= d6) {
    out[0] = t[6]; out[1] = t[7]; out[2] = t[8];
    return;
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    const double s = d2 / (d2 - d6);
    out[0] = a0 + s * ac0; out[1] = a1 + s * ac1; out[2] = a2 + s * ac2;
    return;
  }
  const double va = d3 * d6 - d5 * d4;
  const double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    const double s = e43 / (e43 + e56);
    out[0] = t[3] + s * (t[6] - t[3]);
    out[1] = t[4] + s * (t[7] - t[4]);
    out[2] = t[5] + s * (t[8] - t[5]);
    return;
  }
  const double inv = 1.0 / ((va + vb) + vc);
  const double bv = vb * inv, bw = vc * inv;
  out[0] = (a0 + ab0 * bv) + ac0 * bw;
  out[1] = (a1 + ab1 * bv) + ac1 * bw;
  out[2] = (a2 + ab2 * bv) + ac2 * bw;
}

// Closest point of segment (a, b) to p: the projection parameter, clamped to
// the segment (Ericson Sec. 5.1.2).  A zero-length segment gives a.
__device__ __forceinline__ void closest_on_segment(const double p[3], const double* t,
                                                   double out[3]) {
#pragma clang fp contract(off)
  const double a0 = t[0], a1 = t[1], a2 = t[2];
  const double ab0 = t[3] - a0, ab1 = t[4] - a1, ab2 = t[5] - a2;
  const double u = ((p[0] - a0) * ab0 + (p[1] - a1) * ab1) + (p[2] - a2) * ab2;
  if (u <= 0.0) {
    out[0] = a0; out[1] = a1; out[2] = a2;
    return;
  }
  const double ll = (ab0 * ab0 + ab1 * ab1) + ab2 * ab2;
  if (u >= ll) {
    out[0] = t[3]; out[1] = t[4]; out[2] = t[5];
    return;
  }
  const double f = u / ll;
  out[0] = a0 + f * ab0; out[1] = a1 + f * ab1; out[2] = a2 + f * ab2;
}

// Closest point of the rectangle with corner a = t[0..2] and the two
// neighbouring corners b = t[3..5], d = t[6..8] (orthogonal edges): the
// coordinates of p - a along each edge, clamped to the edge one at a time
// (Ericson Sec. 5.1.4).
__device__ __forceinline__ void closest_on_rectangle(const double p[3], const double* t,
                                                     double out[3]) {
#pragma clang fp contract(off)
  const double a0 = t[0], a1 = t[1], a2 = t[2];
  const double e0 = t[3] - a0, e1 = t[4] - a1, e2 = t[5] - a2;
  const double g0 = t[6] - a0, g1 = t[7] - a1, g2 = t[8] - a2;
  const double q0 = p[0] - a0, q1 = p[1] - a1, q2 = p[2] - a2;
  const double se = (q0 * e0 + q1 * e1) + q2 * e2, le = (e0 * e0 + e1 * e1) + e2 * e2;
  const double sg = (q0 * g0 + q1 * g1) + q2 * g2, lg = (g0 * g0 + g1 * g1) + g2 * g2;
  const double ce = se >= le ? 1.0 : (se > 0.0 ? se / le : 0.0);
  const double cg = sg >= lg ? 1.0 : (sg > 0.0 ? sg / lg : 0.0);
  out[0] = (a0 + ce * e0) + cg * g0;
  out[1] = (a1 + ce * e1) + cg * g1;
  out[2] = (a2 + ce * e2) + cg * g2;
}

// Closest point of mesh element m with nv = 1..4 vertices (point, segment,
// triangle, rectangle; Section 3.3, Fig. 4A-D).  Nine doubles per element:
// the vertex (point), the two ends (segment), the three corners (triangle),
// or corners 0, 1 and 3 of a rectangle (corner 2 is implied).
__device__ __forceinline__ void closest_on_element(const double p[3], const double* t, int nv,
                                                   double out[3]) {
  if (nv == 3) {
    closest_on_triangle(p, t, out);
  } else if (nv == 4) {
    closest_on_rectangle(p, t, out);
  } else if (nv == 2) {
    closest_on_segment(p, t, out);
  } else {
    out[0] = t[0]; out[1] = t[1]; out[2] = t[2];
  }
}

// Host launchers (kernels live in the .hip files).
// Phases of a step as timed by sdem_step_profiled: grid, sort+reorder (+mesh),
// step opening (k_begin), the step kernel (narrow phase, contact law,
// integration), and an empty fifth phase.
constexpr int kPhases = 5;
constexpr int kEvents = kPhases + 3;  // phase boundaries, then the step kernel's own pair
// Spawn attempts of one step (Section 3.1) on the state A at the start of
// the step, before its broad phase: new particles go to slots n.. of A, with
// no contacts in cold; the counters tell how many.
hipError_t launch_spawn(const Ctx& c, const State& A, const Contacts& cold, hipStream_t s);
hipError_t launch_mesh_now(const Ctx& c, hipStream_t s);
hipError_t launch_scatter_radii(const Ctx& c, const State& S, double* R, hipStream_t s);
hipError_t launch_step(const Ctx& c, const State& A, const State& B, const State& T,
                       const Contacts& cold, const Contacts& cnew, int precision, int rebuild,
                       hipStream_t s, hipEvent_t* ev = nullptr);
hipError_t launch_scatter_state(const Ctx& c, const State& S, double* x, double* v, double* w,
                                double* q, double* F, double* T, hipStream_t s);
hipError_t launch_bbox(const Ctx& c, const State& S, hipStream_t s);
hipError_t launch_pack_state(const Ctx& c, const State& S, const double* x, const double* v,
                             const double* w, const double* q, const double* R, hipStream_t s);
hipError_t launch_mesh_planes(const Ctx& c, hipStream_t s);
hipError_t launch_mesh_bins(const Ctx& c, hipStream_t s);
hipError_t launch_selftest(int64_t n, const double* in, const double* in2, double* out,
                           hipStream_t s);
// copies the owned-contact segments of cn (off, cnt) into the records of S
hipError_t launch_set_segments(const Ctx& c, const State& S, const Contacts& cn, hipStream_t s);

}  // namespace sdem
