// Host side of the sdem C ABI: argument checks, workspace carving, parameter
// derivation, step sequencing (HIP graphs of two steps), and reads.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <string>
#include <vector>

#include "sdem_internal.h"

using namespace sdem;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(SDEM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                             \
  } while (0)

constexpr double kPiHost = 3.14159265358979323846;
constexpr int kMaxSimsHost = 4096;

struct Layout {
  size_t total = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    total = (total + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + total) : nullptr;
    total += count * sizeof(T);
    return p;
  }
};

int64_t nwaves_max(const sdem_config& c) { return (c.n_max + kWave - 1) / kWave + 1; }
int64_t nchunks_max(const sdem_config& c) { return nwaves_max(c) + c.nsims_max; }

// Triangle bin tables sized from tri_max: 32 bins and 256 (bin, triangle)
// entries per triangle, within fixed ceilings.
int64_t bins_cap(const sdem_config& c) {
  return c.tri_max > 0 ? std::min<int64_t>(std::max<int64_t>(4096, 32 * c.tri_max), 1 << 22) : 0;
}
int64_t bin_entries_cap(const sdem_config& c) {
  return c.tri_max > 0 ? std::min<int64_t>(256 * c.tri_max + 4096, 1 << 27) : 0;
}

}  // namespace

// Steps that keep the cells run eight to a graph while the rebuild period has
// room for eight; a drift past half the skin inside such a run widens the
// searches of its remaining steps (the contact set stays exact) and halves
// the period at its end.  Contexts from this many particles run their kept
// steps one at a time and look at the drift flag of each (a step there
// takes milliseconds), so that a drift is followed by a rebuild two steps
// later (the flag is read without waiting for the step just queued), unless
// the last whole period saw no drift: then they too run eight to a graph.
constexpr int64_t kDriftCheckEachStep = int64_t(1) << 20;

struct sdem_ctx {
  Ctx c{};
  State st[3]{};  // st[cur] holds the state; st[2] the sorted copy of a rebuild
  Contacts ct[2]{};
  int cur = 0;  // buffer holding the current state and the last step's contacts
  hipStream_t stream = nullptr;
  sdem_config cfg{};
  int nsims = 0;
  int64_t n = 0;
  bool failed = false;
  bool stepped = false;
  double* scratch = nullptr;  // [19][n] for reads into host memory
  std::vector<sdem_params> params;
  std::vector<int64_t> offsets;
  std::vector<std::vector<double>> mesh_tri, mesh_r;  // 9 doubles and R_m per element
  std::vector<std::vector<int32_t>> mesh_nv;          // vertices per element
  std::vector<std::vector<int32_t>> mesh_grp;         // motion group per element
  std::vector<std::vector<MeshMotion>> motion;        // motion groups per simulation
  std::vector<double> rmax;
  // graphs by pattern and starting buffer parity: two full steps, one full
  // step, one step keeping the cells, eight steps keeping the cells
  hipGraphExec_t graph[4][2] = {};
  bool graph_failed = false;
  int64_t graphs_made = 0;  // graphs instantiated so far
  // rebuild schedule (skin > 0): steps since the last rebuild, and a drift
  // past half the skin seen at the last synchronisation (or no rebuild yet)
  int64_t since = 0;
  bool need_rebuild = true;
  int rebuild_every = 1;  // the configured longest period
  int period = 1;         // the current period: halved after a period in which
                          // searches had to reach past the skin, doubled
                          // (up to rebuild_every) after one without
  bool quiet = false;     // the last whole period saw no such drift
  // drift flags of kept steps run one at a time in large contexts: copied to
  // pinned host memory behind each such step and read two steps later, so
  // the host never waits for the step it has just queued
  int32_t* lag_host = nullptr;  // [2]
  hipEvent_t lag_ev[2] = {};
  bool lag_valid[2] = {};
  int lag_slot = 0;
  ~sdem_ctx() {
    for (auto& e : lag_ev)
      if (e) (void)hipEventDestroy(e);
    if (lag_host) (void)hipHostFree(lag_host);
  }
  // particle spawning (one simulation per context)
  bool spawn_on = false;
  SpawnParams spawn{};
  std::vector<int32_t> wchunk_host;  // first chunk of each wave (one simulation: the wave)
  int32_t chunk_end = 0;
};

// Graphs bake the context by value: drop them when a field of it changes.
static void drop_graphs(sdem_ctx* X) {
  for (auto& row : X->graph)
    for (auto& g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// contacts one particle may have in a step (0 selects 64)
static int32_t hit_cap_of(const sdem_config& cfg) {
  return cfg.contacts_per_particle ? cfg.contacts_per_particle : 64;
}

// contact records are allocated per group of kGroup slots: gcap each
static int64_t groups_of(const sdem_config& cfg) {
  return (std::max<int64_t>(cfg.n_max, 1) + kGroup - 1) / kGroup;
}
static int64_t group_cap(const sdem_config& cfg) {
  return std::max<int64_t>(1, (cfg.contacts_max + groups_of(cfg) - 1) / groups_of(cfg));
}

static Layout carve(const sdem_config& cfg, char* base, Ctx* c, State st[2], Contacts ct[2],
                    double** scratch) {
  Layout L;
  L.base = base;
  const size_t N = (size_t)std::max<int64_t>(cfg.n_max, 1);
  const size_t G = (size_t)groups_of(cfg);
  const size_t Cm = G * (size_t)group_cap(cfg);
  const size_t Gm = (size_t)std::max<int64_t>(cfg.cells_max, 1);
  const size_t M = (size_t)std::max<int64_t>(cfg.tri_max, 1);
  const size_t S = (size_t)std::max<int32_t>(cfg.nsims_max, 1);
  const size_t NC = (size_t)nchunks_max(cfg);
  Ctx cc{};
  cc.ctr = L.take<Counters>(1);
  cc.spawn = L.take<SpawnParams>(1);
  cc.spawn_cand = L.take<double4>(kSpawnMax);
  cc.spawn_thr = L.take<unsigned long long>(kSpawnMax);
  cc.sp = L.take<SimParams>(S);
  cc.sg = L.take<SimGrid>(S);
  cc.sim_of = L.take<int32_t>(N);
  cc.wchunk = L.take<int32_t>((size_t)nwaves_max(cfg));
  cc.chunk0 = L.take<int32_t>(S + 1);
  cc.part = L.take<double>(kPart * NC);
  cc.cell_cnt = L.take<int32_t>(Gm);
  cc.cell_start = L.take<int32_t>(Gm + 1);
  cc.key_tmp = L.take<int32_t>(N);
  cc.rank = L.take<int32_t>(N);
  cc.perm = L.take<int32_t>(N);
  cc.scan_tmp = L.take<int32_t>(kScanBlocks + 1);
  cc.gcnt = L.take<int32_t>(G);
  cc.gstat = L.take<unsigned long long>(2 * G);
  cc.xtra = L.take<double>(S);
  cc.spill = L.take<int32_t>(std::max<size_t>(N * (size_t)(hit_cap_of(cfg) - kHit), 1));
  cc.xb = L.take<double4>(N);
  {
    // candidate lists of the particles, kept between rebuilds (skin > 0)
    const size_t NL = cfg.skin > 0.0 ? N : 1;
    cc.vcnt = L.take<int32_t>(NL);
    cc.vlist = L.take<int32_t>(NL * kCand);
    cc.vstride = (int64_t)NL;
  }
  cc.F = L.take<double>(3 * N);
  cc.T = L.take<double>(3 * N);
  cc.tri_ref = L.take<double>(9 * M);
  cc.tri = L.take<double>(9 * M);
  cc.tri_pl = L.take<double>(4 * M);
  cc.rmesh = L.take<double>(M);
  cc.tri_sim = L.take<int32_t>(M);
  cc.tri_nv = L.take<int32_t>(M);
  cc.tri_grp = L.take<int32_t>(M);
  cc.tri_mv = L.take<double>(9 * M);
  cc.frame = L.take<double>(12 * S);
  cc.motion = L.take<MeshMotion>(S * kMotionMax);
  cc.mg = L.take<MeshGrid>(S);
  cc.bin_cnt = L.take<int32_t>((size_t)std::max<int64_t>(bins_cap(cfg), 1));
  cc.bin_start = L.take<int32_t>((size_t)bins_cap(cfg) + 1);
  cc.bin_tri = L.take<int32_t>((size_t)std::max<int64_t>(bin_entries_cap(cfg), 1));
  // two state buffers that alternate every step, and a third for the sorted
  // copy on steps that rebuild the cells
  for (int b = 0; b < 3; ++b) {
    State s{};
    s.xr = L.take<double4>(N);
    s.a = L.take<Aux>(N);
    s.q = L.take<double4>(N);
    if (st) st[b] = s;
  }
  for (int b = 0; b < 2; ++b) {
    Contacts k{};
    k.cnt = L.take<int32_t>(N);
    k.off = L.take<int32_t>(N);
    k.a = L.take<int32_t>(2 * Cm);
    k.b = L.take<int32_t>(2 * Cm);
    k.ref = L.take<int32_t>(Cm);
    k.key = L.take<int2>(Cm);
    k.spr = L.take<double>(kSpr * Cm);
    k.ng = L.take<int32_t>(G);
    if (ct) ct[b] = k;
  }
  double* scr = L.take<double>(19 * N);
  if (scratch) *scratch = scr;
  L.total = (L.total + 255) & ~size_t(255);
  if (c) *c = cc;
  return L;
}

static int check_config(const sdem_config* cfg) {
  if (!cfg) return fail(SDEM_EINVAL, "config is NULL");
  if (cfg->n_max < 0 || cfg->n_max > 0x3fffffff) return fail(SDEM_EINVAL, "n_max out of range");
  if (cfg->contacts_max < 0 || cfg->contacts_max > 0x3fffffff)
    return fail(SDEM_EINVAL, "contacts_max out of range");
  if (groups_of(*cfg) * group_cap(*cfg) > 0x7fffffffLL)
    return fail(SDEM_EINVAL, "contacts_max too large");
  if (cfg->cells_max < 1 || cfg->cells_max > 0x3fffffff)
    return fail(SDEM_EINVAL, "cells_max out of range");
  if (cfg->tri_max < 0 || cfg->tri_max > 0x3fffffff) return fail(SDEM_EINVAL, "tri_max out of range");
  if (cfg->nsims_max < 1 || cfg->nsims_max > kMaxSimsHost)
    return fail(SDEM_EINVAL, "nsims_max must be in [1, %d]", kMaxSimsHost);
  if (cfg->precision != SDEM_FP64 && cfg->precision != SDEM_MIXED)
    return fail(SDEM_EINVAL, "unknown precision %d", cfg->precision);
  if (cfg->block != 0 && (cfg->block < 64 || cfg->block > 1024 || cfg->block % 64))
    return fail(SDEM_EINVAL, "block must be a multiple of 64 in [64, 1024]");
  if (cfg->detect_lanes != 0 && cfg->detect_lanes != 1)
    return fail(SDEM_EINVAL, "detect_lanes must be 0 or 1 (one lane per particle)");
  if (cfg->contacts_per_particle != 0 &&
      (cfg->contacts_per_particle < kMinHitCap || cfg->contacts_per_particle > 4096))
    return fail(SDEM_EINVAL, "contacts_per_particle must be 0 or in [%d, 4096]", kMinHitCap);
  if (!(cfg->cell_factor == 0.0 || cfg->cell_factor >= 0.125) || !isfinite(cfg->cell_factor))
    return fail(SDEM_EINVAL, "cell_factor must be >= 0.125 (0 selects 1)");
  if (!(cfg->skin >= 0.0) || !(cfg->skin <= 100.0))
    return fail(SDEM_EINVAL, "skin must be in [0, 100]");
  if (cfg->rebuild_every < 0) return fail(SDEM_EINVAL, "rebuild_every must be >= 0");
  return SDEM_OK;
}

static int check_params(const sdem_params& p, int s) {
  // Table 2 "Requirements"
  if (!(p.rho > 0) || !(p.E > 0) || !isfinite(p.rho) || !isfinite(p.E))
    return fail(SDEM_EINVAL, "sim %d: rho and E must be > 0", s);
  if (!(p.nu > -1.0 && p.nu <= 0.5)) return fail(SDEM_EINVAL, "sim %d: nu must be in (-1, 0.5]", s);
  if (!(p.e_n >= 0.0 && p.e_n <= 1.0)) return fail(SDEM_EINVAL, "sim %d: e_n must be in [0, 1]", s);
  if (!(p.mu_s >= 0) || !(p.mu_r >= 0) || !(p.mu_t >= 0) || !isfinite(p.mu_s) ||
      !isfinite(p.mu_r) || !isfinite(p.mu_t))
    return fail(SDEM_EINVAL, "sim %d: friction coefficients must be >= 0", s);
  if (!(p.eta >= 0) || !isfinite(p.eta)) return fail(SDEM_EINVAL, "sim %d: eta must be >= 0", s);
  if (!(p.dt > 0) || !isfinite(p.dt)) return fail(SDEM_EINVAL, "sim %d: dt must be > 0", s);
  for (int k = 0; k < 3; ++k)
    if (!isfinite(p.g[k]) || !isfinite(p.mesh_omega[k]) || !isfinite(p.mesh_center[k]))
      return fail(SDEM_EINVAL, "sim %d: g, mesh_omega, mesh_center must be finite", s);
  return SDEM_OK;
}

static bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
         a.type == hipMemoryTypeUnified;
}

static SimParams derive(const sdem_params& p, double cell_factor, double rmax, double skin = 0.0) {
  SimParams d{};
  d.rho = p.rho;
  d.E = p.E;
  d.nu = p.nu;
  d.e_n = p.e_n;
  d.mu_s = p.mu_s;
  d.mu_r = p.mu_r;
  d.mu_t = p.mu_t;
  d.eta = p.eta;
  for (int k = 0; k < 3; ++k) {
    d.g[k] = p.g[k];
  }
  d.dt = p.dt;
  const double r = kPiHost / log(p.e_n);  // e_n = 1 -> inf -> beta 0; e_n = 0 -> beta 1
  d.beta = 1.0 / sqrt(1.0 + r * r);
  const double E = p.E, nu = p.nu;
  d.Es_pp = E / (2.0 * (1.0 - nu * nu));
  d.Gs_pp = E / (4.0 * (2.0 - nu) * (1.0 + nu));
  d.Es_pw = E / (1.0 - nu * nu);
  d.Gs_pw = E / (2.0 * (1.0 + nu) * (2.0 - nu));
  // c_n = sqrt(5 m* k_n) beta with k_n = 4/3 E* a; c_s = sqrt(m* k_s / 6) beta
  // with k_s = 8 G* a (Eq. cn, cs)
  d.cnf_pp = d.beta * sqrt(20.0 / 3.0 * d.Es_pp);
  d.csf_pp = d.beta * sqrt(4.0 / 3.0 * d.Gs_pp);
  d.cnf_pw = d.beta * sqrt(20.0 / 3.0 * d.Es_pw);
  d.csf_pw = d.beta * sqrt(4.0 / 3.0 * d.Gs_pw);
  // cell edge >= 2 R_max; the small margin keeps neighbours within one cell
  // index of each other despite rounding of the cell coordinate
  const double rm = rmax > 0 ? rmax : 1.0;
  d.rmax = rm;
  d.h = cell_factor * 2.0 * rm;
  d.half_skin = 0.5 * skin * rm;
  return d;
}

// The motion of a simulation's mesh given by its parameters alone: one group
// turning with mesh_omega about mesh_center.
static MeshMotion default_motion(const sdem_params& p) {
  MeshMotion g{};
  for (int k = 0; k < 3; ++k) {
    g.omega[k] = p.mesh_omega[k];
    g.center[k] = p.mesh_center[k];
  }
  g.moving = (p.mesh_omega[0] != 0.0 || p.mesh_omega[1] != 0.0 || p.mesh_omega[2] != 0.0);
  return g;
}

// Every element of the mesh in the same motion group.
static bool one_motion_group(const std::vector<int32_t>& grp) {
  for (int32_t g : grp)
    if (g != grp[0]) return false;
  return !grp.empty();
}

static int upload_params(sdem_ctx* x) {
  std::vector<SimParams> sp(x->nsims);
  int tri0 = 0;
  for (int s = 0; s < x->nsims; ++s) {
    sp[s] = derive(x->params[s], x->cfg.cell_factor, x->rmax[s], x->cfg.skin);
    sp[s].p0 = (int32_t)x->offsets[s];
    sp[s].np = (int32_t)(x->offsets[s + 1] - x->offsets[s]);
    sp[s].tri0 = tri0;
    sp[s].ntri = (int32_t)x->mesh_r[s].size();
    tri0 += sp[s].ntri;
  }
  x->c.any_moving = 0;
  x->c.rebin = 0;
  for (int s = 0; s < x->nsims; ++s) {
    sp[s].moving = 0;
    for (size_t m = 0; m < x->mesh_grp[s].size(); ++m)
      if (x->motion[s][x->mesh_grp[s][m]].moving) sp[s].moving = 1;
    sp[s].frame_bins = sp[s].moving && one_motion_group(x->mesh_grp[s]) ? 1 : 0;
    if (sp[s].moving) x->c.any_moving = 1;
    if (sp[s].moving && !sp[s].frame_bins) x->c.rebin = 1;
  }
  HIP_TRY(hipMemcpyAsync(x->c.sp, sp.data(), sizeof(SimParams) * x->nsims, hipMemcpyHostToDevice,
                         x->stream));
  HIP_TRY(hipStreamSynchronize(x->stream));
  return SDEM_OK;
}

namespace sdem {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace sdem

// Device scratch for sdem_init_static (callers that cannot allocate): one
// array per device, held until the process ends.  In host code `scratch` only
// stands for the symbol; its device address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = size_t(SDEM_STATIC_SCRATCH_BYTES);
constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static void* g_scratch_ptr[kMaxStaticDevices] = {};

static void* static_scratch_of(int dev) {
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(SDEM_EHIP, "hipGetSymbolAddress of the static scratch failed: %s",
           hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

extern "C" {

size_t sdem_workspace_bytes(const sdem_config* cfg) {
  if (check_config(cfg) != SDEM_OK) return 0;
  return carve(*cfg, nullptr, nullptr, nullptr, nullptr, nullptr).total;
}

int sdem_init_batch(sdem_ctx** out, const sdem_config* cfg_in, int32_t nsims,
                    const sdem_params* params, const int64_t* offsets, const double* x,
                    const double* v, const double* w, const double* q, const double* R,
                    void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return fail(SDEM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_config(cfg_in);
  if (rc) return rc;
  sdem_config cfg = *cfg_in;
  if (cfg.cell_factor == 0.0) cfg.cell_factor = 1.0;
  if (cfg.block == 0) cfg.block = kThreads;
  cfg.contacts_per_particle = hit_cap_of(cfg);
  if (nsims < 1 || nsims > cfg.nsims_max)
    return fail(SDEM_ECAPACITY, "nsims %d outside [1, nsims_max=%d]", nsims, cfg.nsims_max);
  if (!params || !offsets) return fail(SDEM_EINVAL, "params and offsets are required");
  if (offsets[0] != 0) return fail(SDEM_EINVAL, "offsets[0] must be 0");
  for (int s = 0; s < nsims; ++s) {
    if (offsets[s + 1] < offsets[s]) return fail(SDEM_EINVAL, "offsets must be non-decreasing");
    if ((rc = check_params(params[s], s))) return rc;
  }
  const int64_t n = offsets[nsims];
  if (n > cfg.n_max) return fail(SDEM_ECAPACITY, "n = %lld exceeds n_max = %lld", (long long)n,
                                 (long long)cfg.n_max);
  if (n > 0 && (!x || !R)) return fail(SDEM_EINVAL, "x and R are required");
  const size_t need = sdem_workspace_bytes(&cfg);
  if (!workspace || ws_bytes < need)
    return fail(SDEM_ECAPACITY, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(SDEM_EINVAL, "workspace must be 256-byte aligned");

  // radii: validate and find each simulation's largest (cell edge, Section 3.3)
  std::vector<double> Rh((size_t)n);
  if (n) {
    HIP_TRY(hipMemcpy(Rh.data(), R, sizeof(double) * n, hipMemcpyDefault));
  }
  std::vector<double> rmax(nsims, 0.0);
  for (int s = 0; s < nsims; ++s)
    for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) {
      if (!(Rh[i] > 0) || !isfinite(Rh[i]))
        return fail(SDEM_EINVAL, "radius %lld is not a positive finite number", (long long)i);
      rmax[s] = std::max(rmax[s], Rh[i]);
    }

  sdem_ctx* X = new sdem_ctx();
  X->cfg = cfg;
  X->nsims = nsims;
  X->n = n;
  X->stream = reinterpret_cast<hipStream_t>(hip_stream);
  X->params.assign(params, params + nsims);
  X->offsets.assign(offsets, offsets + nsims + 1);
  X->mesh_tri.assign(nsims, {});
  X->mesh_r.assign(nsims, {});
  X->mesh_nv.assign(nsims, {});
  X->mesh_grp.assign(nsims, {});
  X->motion.resize(nsims);
  for (int s = 0; s < nsims; ++s) X->motion[s].assign(1, default_motion(params[s]));
  X->rmax = rmax;
  carve(cfg, reinterpret_cast<char*>(workspace), &X->c, X->st, X->ct, &X->scratch);
  Ctx& c = X->c;
  c.n = (int32_t)n;
  c.nsims = nsims;
  c.ntri = 0;
  c.cap_contacts = (int32_t)cfg.contacts_max;
  c.cap_cells = (int32_t)cfg.cells_max;
  c.hit_cap = hit_cap_of(cfg);
  c.skin_on = cfg.skin > 0.0 ? 1 : 0;
  X->rebuild_every = c.skin_on ? (cfg.rebuild_every > 0 ? cfg.rebuild_every : 64) : 1;
  X->period = X->rebuild_every;
  if (c.skin_on && cfg.n_max >= kDriftCheckEachStep) {
    void* h = nullptr;
    if (hipHostMalloc(&h, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
      delete X;
      return fail(SDEM_EHIP, "pinned host memory for the drift flags: %s",
                  hipGetErrorString(hipGetLastError()));
    }
    X->lag_host = static_cast<int32_t*>(h);
    for (auto& e : X->lag_ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        delete X;
        return fail(SDEM_EHIP, "drift flag events");
      }
  }
  c.ngroups = (int32_t)((std::max<int64_t>(n, 1) + kGroup - 1) / kGroup);
  c.gcap = (int32_t)group_cap(cfg);

  auto bail = [&](int code) {
    delete X;
    return code;
  };
  hipStream_t st = X->stream;
  // per-slot simulation id; bounding-box chunks = (wave of 64 slots,
  // simulation) segments, in slot order (so simulations ascend)
  std::vector<int32_t> sim_of((size_t)std::max<int64_t>(n, 1)), chunk0(nsims + 1);
  std::vector<int32_t> wchunk((size_t)std::max<int64_t>((n + kWave - 1) / kWave, 1), 0), chunk_sim;
  for (int s = 0; s < nsims; ++s)
    for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) sim_of[i] = s;
  for (int64_t w = 0; w * kWave < n; ++w) {
    wchunk[w] = (int32_t)chunk_sim.size();
    int prev = -1;
    for (int64_t i = w * kWave; i < std::min<int64_t>(n, (w + 1) * kWave); ++i)
      if (sim_of[i] != prev) {
        prev = sim_of[i];
        chunk_sim.push_back(prev);
      }
  }
  for (int s = 0; s <= nsims; ++s)
    chunk0[s] = (int32_t)(std::lower_bound(chunk_sim.begin(), chunk_sim.end(), s) - chunk_sim.begin());
  c.nchunks = (int32_t)chunk_sim.size();

  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, st) : hipSuccess;
  };
  // caller arrays that are not device memory are staged through the scratch
  const double* in[5] = {x, v, w, q, R};
  const size_t words[5] = {3, 3, 3, 4, 1};
  const double* dev_in[5];
  hipError_t e = hipSuccess;
  size_t at = 0;
  for (int k = 0; k < 5 && !e; ++k) {
    dev_in[k] = nullptr;
    if (in[k] && n) {
      if (is_device_ptr(in[k])) {
        dev_in[k] = in[k];
      } else {
        double* d = X->scratch + at * n;
        e = cp(d, in[k], sizeof(double) * words[k] * n);
        dev_in[k] = d;
      }
    }
    at += words[k];
  }
  if (!e) e = hipMemsetAsync(c.ctr, 0, sizeof(Counters), st);
  if (!e) e = hipMemsetAsync(c.cell_cnt, 0, sizeof(int32_t) * cfg.cells_max, st);
  for (int b = 0; b < 2 && !e; ++b) {
    e = hipMemsetAsync(X->ct[b].cnt, 0, sizeof(int32_t) * std::max<int64_t>(n, 1), st);
    if (!e) e = hipMemsetAsync(X->ct[b].off, 0, sizeof(int32_t) * std::max<int64_t>(n, 1), st);
    if (!e) e = hipMemsetAsync(X->ct[b].ng, 0, sizeof(int32_t) * groups_of(cfg), st);
  }
  if (!e) e = hipMemsetAsync(c.gcnt, 0, sizeof(int32_t) * c.ngroups, st);
  if (!e) e = hipMemsetAsync(c.gstat, 0, sizeof(unsigned long long) * 2 * c.ngroups, st);
  if (!e) e = cp(c.sim_of, sim_of.data(), sizeof(int32_t) * n);
  if (!e) e = cp(c.wchunk, wchunk.data(), sizeof(int32_t) * wchunk.size());
  if (!e) e = cp(c.chunk0, chunk0.data(), sizeof(int32_t) * chunk0.size());
  if (!e) e = launch_pack_state(c, X->st[0], dev_in[0], dev_in[1], dev_in[2], dev_in[3],
                                dev_in[4], st);
  // bounding-box partials of the initial state (each step's integration
  // writes those of the next)
  if (!e) e = launch_bbox(c, X->st[0], st);
  if (!e) e = hipStreamSynchronize(st);
  if (e) {
    fail(SDEM_EHIP, "init copies failed: %s", hipGetErrorString(e));
    return bail(SDEM_EHIP);
  }
  if ((rc = upload_params(X))) return bail(rc);
  *out = X;
  return SDEM_OK;
}

int sdem_init(sdem_ctx** out, const sdem_config* cfg, const sdem_params* params, int64_t n,
              const double* x, const double* v, const double* w, const double* q,
              const double* R, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (n < 0) return fail(SDEM_EINVAL, "n must be >= 0");
  const int64_t off[2] = {0, n};
  return sdem_init_batch(out, cfg, 1, params, off, x, v, w, q, R, workspace, ws_bytes,
                         hip_stream);
}

int sdem_init_static(sdem_ctx** out, const sdem_config* cfg, const sdem_params* params,
                     int64_t n, const double* x, const double* v, const double* w,
                     const double* q, const double* R, void* hip_stream) {
  if (!out) return fail(SDEM_EINVAL, "out is NULL");
  *out = nullptr;
  if (check_config(cfg) != SDEM_OK) return SDEM_EINVAL;
  const size_t need = sdem_workspace_bytes(cfg);
  if (need > kStaticScratchBytes)
    return fail(SDEM_ECAPACITY,
                "these capacities need %zu bytes of workspace; the static scratch holds %zu "
                "(use sdem_init with a workspace of your own)",
                need, kStaticScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices)
    return fail(SDEM_EINVAL, "device %d: the static scratch serves devices 0..%d", dev,
                kMaxStaticDevices - 1);
  void* ptr = static_scratch_of(dev);
  if (!ptr) return SDEM_EHIP;  // message set by static_scratch_of
  return sdem_init(out, cfg, params, n, x, v, w, q, R, ptr, kStaticScratchBytes, hip_stream);
}

// Corners of element m (its stored vertices, plus the implied fourth corner
// of a rectangle); returns their number.
static int element_corners(const std::vector<double>& tri, const std::vector<int32_t>& nv,
                           size_t m, double out[4][3]) {
  const double* t = tri.data() + 9 * m;
  for (int v = 0; v < 3; ++v)
    for (int a = 0; a < 3; ++a) out[v][a] = t[3 * v + a];
  if (nv[m] != 4) return 3;
  for (int a = 0; a < 3; ++a) out[3][a] = (t[3 + a] + t[6 + a]) - t[a];
  return 4;
}

// Bin grid of one simulation's mesh.  The grid spans every place the
// elements can reach (fixed, vibrating or turning), grown by
// reach = rmax + max R_m, where rmax is the simulation's R_max plus the half
// skin (a rebuild records the elements within R_i + R_m + half skin).  The bin edge starts at the larger of 2 reach and
// half the median element extent and grows until the bins, and a bound on
// the (bin, element) entries that holds at any orientation, fit this
// simulation's share of the tables.
static MeshGrid mesh_grid(const std::vector<double>& tri, const std::vector<int32_t>& nv,
                          const std::vector<double>& rm, const std::vector<int32_t>& grp,
                          const std::vector<MeshMotion>& motion, double rmax, int64_t bins_budget,
                          int64_t entries_budget, int32_t off) {
  MeshGrid G{};
  const size_t nt = rm.size();
  double rmesh_max = 0.0;
  for (double r : rm) rmesh_max = std::max(rmesh_max, r);
  const double reach = (rmax + rmesh_max) * (1.0 + 1e-6);
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = HUGE_VAL;
    hi[a] = -HUGE_VAL;
  }
  // every place an element's corners can reach: a ball about the rotation
  // centre for a turning group, the box grown by twice the amplitude for a
  // vibrating one (|sin - sin phase| <= 2), the box itself for a fixed one
  for (size_t m = 0; m < nt; ++m) {
    const MeshMotion& g = motion[grp[m]];
    double cr[4][3];
    const int k = element_corners(tri, nv, m, cr);
    double sw[3];
    for (int a = 0; a < 3; ++a) sw[a] = g.moving ? 2.0 * fabs(g.amp[a]) : 0.0;
    const bool turns = g.omega[0] != 0.0 || g.omega[1] != 0.0 || g.omega[2] != 0.0;
    for (int v = 0; v < k; ++v) {
      if (turns) {
        const double dx = cr[v][0] - g.center[0], dy = cr[v][1] - g.center[1],
                     dz = cr[v][2] - g.center[2];
        const double rv = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 1e-9);
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], g.center[a] - (rv + sw[a] + reach));
          hi[a] = std::max(hi[a], g.center[a] + (rv + sw[a] + reach));
        }
      } else {
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], cr[v][a] - (sw[a] + reach));
          hi[a] = std::max(hi[a], cr[v][a] + (sw[a] + reach));
        }
      }
    }
  }
  double span[3], smax = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double pad = 1e-6 * (hi[a] - lo[a]) + 1e-9 * (fabs(lo[a]) + fabs(hi[a])) + 1e-12;
    lo[a] -= pad;
    hi[a] += pad;
    span[a] = hi[a] - lo[a];
    smax = std::max(smax, span[a]);
  }
  // per element: largest corner distance from the corners' mean (rotation
  // invariant) and largest box edge
  std::vector<double> rb(nt), ext(nt);
  for (size_t m = 0; m < nt; ++m) {
    double cr[4][3];
    const int k = element_corners(tri, nv, m, cr);
    double c3[3], e = 0.0, r = 0.0;
    for (int a = 0; a < 3; ++a) {
      double sum = 0.0, mn = cr[0][a], mx = cr[0][a];
      for (int v = 0; v < k; ++v) {
        sum += cr[v][a];
        mn = std::min(mn, cr[v][a]);
        mx = std::max(mx, cr[v][a]);
      }
      c3[a] = sum / k;
      e = std::max(e, mx - mn);
    }
    for (int v = 0; v < k; ++v) {
      const double dx = cr[v][0] - c3[0], dy = cr[v][1] - c3[1], dz = cr[v][2] - c3[2];
      r = std::max(r, sqrt(dx * dx + dy * dy + dz * dz));
    }
    rb[m] = r * (1.0 + 1e-6) + (rmax + rm[m]) * (1.0 + 1e-6);
    ext[m] = e;
  }
  std::vector<double> es = ext;
  std::nth_element(es.begin(), es.begin() + es.size() / 2, es.end());
  double h = std::max({2.0 * reach, 0.5 * es[es.size() / 2], smax * 1e-6});
  for (int it = 0; it < 400; ++it, h *= 1.25) {
    int64_t dims[3], bins = 1;
    for (int a = 0; a < 3; ++a) {
      dims[a] = (int64_t)floor(span[a] / h) + 1;
      bins *= dims[a];
    }
    if (bins > bins_budget) continue;
    int64_t entries = 0;
    for (size_t m = 0; m < nt && entries <= entries_budget; ++m) {
      int64_t per = 1;
      for (int a = 0; a < 3; ++a) per *= std::min<int64_t>(dims[a], (int64_t)floor(2.0 * rb[m] / h) + 2);
      entries += per;
    }
    if (entries > entries_budget) continue;
    for (int a = 0; a < 3; ++a) {
      G.lo[a] = lo[a];
      G.dim[a] = (int32_t)dims[a];
    }
    G.inv_h = 1.0 / h;
    G.off = off;
    return G;
  }
  G.dim[0] = 0;  // no grid fits (cannot happen for budgets >= 8 per triangle)
  return G;
}

// A rectangle needs a right angle at corner 0 and corner 2 at corner 1 +
// corner 3 - corner 0, each to 1e-6 relative to its edges.
static bool is_rectangle(const double* v) {
  double e[3], g[3], h[3];
  for (int a = 0; a < 3; ++a) {
    e[a] = v[3 + a] - v[a];
    g[a] = v[9 + a] - v[a];
    h[a] = v[6 + a] - ((v[3 + a] + v[9 + a]) - v[a]);
  }
  const double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  const double lg = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const double lh = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  if (fabs(e[0] * g[0] + e[1] * g[1] + e[2] * g[2]) > 1e-6 * le * lg) return false;
  return lh <= 1e-6 * (le + lg);
}

static int upload_mesh(sdem_ctx* X);

// Elements of nv[m] = 1..4 vertices, verts [nel][4][3] (tri != NULL instead
// gives triangles [nel][3][3]).
static int set_mesh(sdem_ctx* X, int32_t sim, int64_t nel, const int32_t* nv, const double* verts,
                    const double* tri, const double* rmesh) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->stepped) return fail(SDEM_ESTATE, "meshes are fixed once stepping has started");
  if (sim < 0 || sim >= X->nsims) return fail(SDEM_EINVAL, "sim %d out of range", sim);
  if (nel < 0 || (nel > 0 && !tri && (!nv || !verts)))
    return fail(SDEM_EINVAL, "bad mesh element arrays");
  std::vector<double> packed((size_t)9 * nel);
  std::vector<int32_t> counts((size_t)nel, 3);
  for (int64_t m = 0; m < nel; ++m) {
    const int k = tri ? 3 : nv[m];
    if (k < 1 || k > 4)
      return fail(SDEM_EINVAL, "element %lld has %d vertices (1..4 allowed)", (long long)m, k);
    const double* v = tri ? tri + 9 * m : verts + 12 * m;
    for (int j = 0; j < 3 * k; ++j)
      if (!isfinite(v[j]))
        return fail(SDEM_EINVAL, "vertex coordinate of element %lld is not finite", (long long)m);
    if (k == 4 && !is_rectangle(v))
      return fail(SDEM_EINVAL, "element %lld is not a rectangle (corners in cyclic order)",
                  (long long)m);
    // stored slots: the vertex three times, the ends and the last end again,
    // the three corners, or corners 0, 1 and 3 of a rectangle
    static const int slots[5][3] = {{0, 0, 0}, {0, 0, 0}, {0, 1, 1}, {0, 1, 2}, {0, 1, 3}};
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) packed[9 * m + 3 * j + a] = v[3 * slots[k][j] + a];
    counts[m] = k;
  }
  for (int64_t m = 0; rmesh && m < nel; ++m)
    if (!(rmesh[m] >= 0) || !isfinite(rmesh[m]))
      return fail(SDEM_EINVAL, "mesh radius %lld must be >= 0", (long long)m);
  int64_t total = nel;
  for (int s = 0; s < X->nsims; ++s)
    if (s != sim) total += (int64_t)X->mesh_r[s].size();
  if (total > X->cfg.tri_max)
    return fail(SDEM_ECAPACITY, "%lld mesh elements exceed tri_max = %lld", (long long)total,
                (long long)X->cfg.tri_max);
  X->mesh_tri[sim] = std::move(packed);
  X->mesh_nv[sim] = std::move(counts);
  X->mesh_grp[sim].assign((size_t)nel, 0);
  X->mesh_r[sim].assign((size_t)nel, 0.0);
  if (rmesh) X->mesh_r[sim].assign(rmesh, rmesh + nel);
  return upload_mesh(X);
}

// Uploads the meshes of every simulation and builds their element bins
// (reach R_max + half skin + R_m of each simulation).
static int upload_mesh(sdem_ctx* X) {
  drop_graphs(X);
  // concatenate every simulation's mesh
  std::vector<double> all, rad;
  std::vector<int32_t> owner, nva, grp;
  std::vector<MeshMotion> table((size_t)X->nsims * kMotionMax);
  for (int s = 0; s < X->nsims; ++s) {
    all.insert(all.end(), X->mesh_tri[s].begin(), X->mesh_tri[s].end());
    rad.insert(rad.end(), X->mesh_r[s].begin(), X->mesh_r[s].end());
    nva.insert(nva.end(), X->mesh_nv[s].begin(), X->mesh_nv[s].end());
    owner.insert(owner.end(), X->mesh_r[s].size(), s);
    for (int32_t g : X->mesh_grp[s]) grp.push_back(s * kMotionMax + g);
    for (size_t g = 0; g < X->motion[s].size(); ++g) table[(size_t)s * kMotionMax + g] = X->motion[s][g];
  }
  Ctx& c = X->c;
  c.ntri = (int32_t)rad.size();
  hipStream_t st = X->stream;
  if (c.ntri) {
    HIP_TRY(hipMemcpyAsync(c.tri_ref, all.data(), sizeof(double) * all.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.rmesh, rad.data(), sizeof(double) * rad.size(), hipMemcpyHostToDevice,
                           st));
    HIP_TRY(hipMemcpyAsync(c.tri_sim, owner.data(), sizeof(int32_t) * owner.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.tri_nv, nva.data(), sizeof(int32_t) * nva.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.tri_grp, grp.data(), sizeof(int32_t) * grp.size(),
                           hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(c.motion, table.data(), sizeof(MeshMotion) * table.size(),
                         hipMemcpyHostToDevice, st));
  int rc = upload_params(X);
  if (rc) return rc;
  // triangle bins: each simulation gets a share of the tables in proportion
  // to its triangles
  std::vector<MeshGrid> mg(X->nsims);
  int64_t nbins = 0;
  const int64_t tmax = std::max<int64_t>(X->cfg.tri_max, 1);
  for (int s = 0; s < X->nsims; ++s) {
    const int64_t nt = (int64_t)X->mesh_r[s].size();
    mg[s] = MeshGrid{};
    mg[s].off = (int32_t)nbins;
    if (!nt) continue;
    const int64_t bb = bins_cap(X->cfg) * nt / tmax, eb = bin_entries_cap(X->cfg) * nt / tmax;
    // the reach of the bins: R_max plus the half skin (as derive() sets it)
    const double rm = X->rmax[s] > 0 ? X->rmax[s] : 1.0;
    const double rreach = rm + 0.5 * X->cfg.skin * rm;
    // a mesh moving as one body is binned once in its own frame: the grid
    // covers its elements at t = 0 only
    std::vector<MeshMotion> still(X->motion[s].size());
    const bool frame = one_motion_group(X->mesh_grp[s]) && X->motion[s][X->mesh_grp[s][0]].moving;
    mg[s] = mesh_grid(X->mesh_tri[s], X->mesh_nv[s], X->mesh_r[s], X->mesh_grp[s],
                      frame ? still : X->motion[s], rreach, std::max<int64_t>(bb, 1), eb,
                      (int32_t)nbins);
    if (mg[s].dim[0] <= 0) return fail(SDEM_ECAPACITY, "no triangle bin grid fits simulation %d", s);
    nbins += (int64_t)mg[s].dim[0] * mg[s].dim[1] * mg[s].dim[2];
  }
  c.nbins = (int32_t)nbins;
  c.cap_bin_entries = (int32_t)bin_entries_cap(X->cfg);
  HIP_TRY(hipMemcpyAsync(c.mg, mg.data(), sizeof(MeshGrid) * X->nsims, hipMemcpyHostToDevice, st));
  if (nbins) HIP_TRY(hipMemsetAsync(c.bin_cnt, 0, sizeof(int32_t) * nbins, st));
  HIP_TRY(launch_mesh_planes(c, st));
  HIP_TRY(launch_mesh_bins(c, st));
  Counters ctr;
  HIP_TRY(hipMemcpyAsync(&ctr, c.ctr, sizeof ctr, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctr.flags & kFlagCapBins) {
    X->failed = true;
    return fail(SDEM_ECAPACITY, "the mesh element bins overflowed their table of %d entries",
                c.cap_bin_entries);
  }
  return SDEM_OK;
}

int sdem_add_mesh(sdem_ctx* X, int32_t sim, int64_t ntri, const double* tri, const double* rmesh) {
  if (ntri > 0 && !tri) return fail(SDEM_EINVAL, "bad triangle array");
  return set_mesh(X, sim, ntri, nullptr, nullptr, ntri > 0 ? tri : nullptr, rmesh);
}

int sdem_add_mesh_elements(sdem_ctx* X, int32_t sim, int64_t nel, const int32_t* nverts,
                           const double* verts, const double* rmesh) {
  return set_mesh(X, sim, nel, nverts, verts, nullptr, rmesh);
}

int sdem_set_history(sdem_ctx* X, int64_t nc, const int32_t* ki, const int32_t* kj,
                     const double* us, const double* ur, const double* ut) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->failed) return fail(SDEM_ESTATE, "context failed in an earlier step");
  if (nc < 0 || (nc > 0 && (!ki || !kj || !us || !ur || !ut)))
    return fail(SDEM_EINVAL, "bad history arrays");
  if (nc > X->cfg.contacts_max)
    return fail(SDEM_ECAPACITY, "%lld history entries exceed contacts_max", (long long)nc);
  const int64_t n = X->n;
  hipStream_t st = X->stream;
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<int32_t> pid((size_t)std::max<int64_t>(n, 1)), slot((size_t)std::max<int64_t>(n, 1));
  if (n)
    HIP_TRY(hipMemcpy2D(pid.data(), sizeof(int32_t), &X->st[X->cur].a[0].pid, sizeof(Aux),
                        sizeof(int32_t), (size_t)n, hipMemcpyDeviceToHost));
  for (int64_t s = 0; s < n; ++s) slot[pid[s]] = (int32_t)s;
  std::vector<int32_t> owner((size_t)nc);
  std::vector<int32_t> simof((size_t)std::max<int64_t>(n, 1));
  for (int s = 0; s < X->nsims; ++s)
    for (int64_t i = X->offsets[s]; i < X->offsets[s + 1]; ++i) simof[i] = s;
  for (int64_t e = 0; e < nc; ++e) {
    if (ki[e] < 0 || ki[e] >= n) return fail(SDEM_EINVAL, "history key %lld: bad ki", (long long)e);
    if (kj[e] > 0) {
      if (kj[e] >= n || kj[e] <= ki[e] || simof[kj[e]] != simof[ki[e]])
        return fail(SDEM_EINVAL, "history key %lld: bad particle pair", (long long)e);
      owner[e] = slot_owns(slot[ki[e]], slot[kj[e]]) ? slot[ki[e]] : slot[kj[e]];
    } else {
      if (-(int64_t)kj[e] >= (int64_t)X->mesh_r[simof[ki[e]]].size())
        return fail(SDEM_EINVAL, "history key %lld: no such triangle", (long long)e);
      owner[e] = slot[ki[e]];
    }
  }
  // group by owner slot (counting sort); records of slot group g start at
  // g * gcap, each owner's records contiguous
  std::vector<int32_t> cnt((size_t)std::max<int64_t>(n, 1), 0), off((size_t)std::max<int64_t>(n, 1), 0);
  for (int64_t e = 0; e < nc; ++e) ++cnt[owner[e]];
  const int64_t gcap = X->c.gcap;
  std::vector<int32_t> used((size_t)X->c.ngroups, 0);
  for (int64_t s = 0; s < n; ++s) {
    const int64_t g = s >> kGroupShift;
    off[s] = (int32_t)(g * gcap + used[g]);
    used[g] += cnt[s];
    if (used[g] > gcap)
      return fail(SDEM_ECAPACITY, "history: slot group %lld needs more than its %lld records",
                  (long long)g, (long long)gcap);
  }
  std::vector<int32_t> pos(off.begin(), off.end());
  const size_t Ctot = (size_t)X->c.ngroups * (size_t)gcap;
  std::vector<int2> K(Ctot);
  std::vector<double> SP((size_t)kSpr * Ctot, 0.0);
  for (int64_t e = 0; e < nc; ++e) {
    const int32_t d = pos[owner[e]]++;
    K[d] = make_int2(ki[e], kj[e]);
    for (int k = 0; k < 3; ++k) {
      SP[(size_t)kSpr * d + k] = us[3 * e + k];
      SP[(size_t)kSpr * d + 3 + k] = ur[3 * e + k];
    }
    SP[(size_t)kSpr * d + 6] = ut[e];
  }
  Contacts& C = X->ct[X->cur];
  HIP_TRY(hipMemcpy(C.ng, used.data(), sizeof(int32_t) * used.size(), hipMemcpyHostToDevice));
  if (n) {
    HIP_TRY(hipMemcpy(C.cnt, cnt.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(C.off, off.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  if (nc) {
    HIP_TRY(hipMemcpy(C.key, K.data(), sizeof(int2) * Ctot, hipMemcpyHostToDevice));
    if (X->cfg.precision == SDEM_MIXED) {
      // the mixed path keeps springs as floats, eight to a record
      std::vector<float> SF(SP.begin(), SP.end());
      HIP_TRY(hipMemcpy(C.spr, SF.data(), sizeof(float) * kSpr * Ctot, hipMemcpyHostToDevice));
    } else {
      HIP_TRY(hipMemcpy(C.spr, SP.data(), sizeof(double) * kSpr * Ctot, hipMemcpyHostToDevice));
    }
  }
  // the particles' records carry their segments for the next step
  HIP_TRY(launch_set_segments(X->c, X->st[X->cur], C, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

// ---------------------------------------------------------------------------
// particle spawning (Section 3.1): one simulation per context
// ---------------------------------------------------------------------------
// The particle count grows from X->n to n1 (the new particles are already in
// slots X->n .. n1-1 of the current state): every count-dependent field of
// the context follows.
static int grow_n(sdem_ctx* X, int64_t n1) {
  const int64_t n0 = X->n;
  Ctx& c = X->c;
  hipStream_t st = X->stream;
  X->n = n1;
  X->offsets[1] = n1;
  c.n = (int32_t)n1;
  c.ngroups = (int32_t)((std::max<int64_t>(n1, 1) + kGroup - 1) / kGroup);
  // one simulation: chunk w is wave w
  const int64_t w0 = (n0 + kWave - 1) / kWave, w1 = (n1 + kWave - 1) / kWave;
  if ((int64_t)X->wchunk_host.size() < w1) X->wchunk_host.resize((size_t)w1);
  for (int64_t w = w0; w < w1; ++w) X->wchunk_host[w] = (int32_t)w;
  X->chunk_end = (int32_t)w1;
  c.nchunks = (int32_t)w1;
  if (w1 > w0)
    HIP_TRY(hipMemcpyAsync(c.wchunk + w0, X->wchunk_host.data() + w0, sizeof(int32_t) * (w1 - w0),
                           hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c.chunk0 + 1, &X->chunk_end, sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (n1 > n0) HIP_TRY(hipMemsetAsync(c.sim_of + n0, 0, sizeof(int32_t) * (n1 - n0), st));
  drop_graphs(X);
  return upload_params(X);  // the simulation's particle range
}

static bool spawning(const sdem_ctx* X) {
  return X->spawn_on && X->spawn.n_spawn > 0 && X->n < X->spawn.n_max;
}

// The spawn attempts of the step about to run; waits for them.  *stop is set
// when an earlier step of the call has failed (the caller reports it).
static int spawn_now(sdem_ctx* X, bool* stop) {
  *stop = false;
  HIP_TRY(launch_spawn(X->c, X->st[X->cur], X->ct[X->cur], X->stream));
  Counters h;
  HIP_TRY(hipMemcpyAsync(&h, X->c.ctr, sizeof h, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if (h.flags) {
    *stop = true;
    return SDEM_OK;
  }
  if (h.rebuild_next) X->need_rebuild = true;
  if (h.spawn_new > 0) {
    const int rc = grow_n(X, X->n + h.spawn_new);
    if (rc) return rc;
    X->need_rebuild = true;  // the new particles need cells
  }
  return SDEM_OK;
}

// After a batch of steps: read the counters, locate a failed step, report.
static int finish_steps(sdem_ctx* X, const Counters& before, int start) {
  Counters after;
  HIP_TRY(hipMemcpyAsync(&after, X->c.ctr, sizeof after, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if (after.rebuild_next) X->need_rebuild = true;
  if (!after.flags) return SDEM_OK;
  const int64_t done = (int64_t)(after.steps - before.steps) - 1;  // the failed one counted
  X->cur = (int)((start + done) & 1);
  X->failed = true;
  const long long at = (long long)(before.steps + done);
  if (after.flags & kFlagCapCells)
    return fail(SDEM_ECAPACITY,
                "step %lld: the grid needs %d cells, cells_max is %lld (particles spread too "
                "far; confine them with a mesh or raise cells_max)",
                at, after.need_cells, (long long)X->cfg.cells_max);
  if (after.flags & kFlagCapContacts)
    return fail(SDEM_ECAPACITY,
                "step %lld: a group of %d particle slots needed %d contact records, its share "
                "of contacts_max = %lld is %d; raise contacts_max",
                at, kGroup, after.need_group, (long long)X->cfg.contacts_max, X->c.gcap);
  if (after.flags & kFlagCapBins)
    return fail(SDEM_ECAPACITY, "step %lld: the triangle bins overflowed their table of %d "
                "entries", at, X->c.cap_bin_entries);
  if (after.flags & kFlagCapPerParticle)
    return fail(SDEM_ECAPACITY,
                "step %lld: a particle has more than contacts_per_particle = %d contacts; "
                "raise contacts_per_particle",
                at, X->c.hit_cap);
  return fail(SDEM_ENONFINITE, "step %lld: non-finite position, velocity or spin", at);
}

// Steps keep the cells when a skin is set, except every rebuild_every-th
// step and the first step after a drift past half the skin was seen.
static bool rebuild_now(const sdem_ctx* X) {
  return !X->c.skin_on || X->need_rebuild || X->since >= X->period;
}
static void count_step(sdem_ctx* X, bool rebuild) {
  if (rebuild) {
    X->since = 1;
    X->need_rebuild = false;
  } else {
    ++X->since;
  }
}

// k steps from the current buffer parity, all rebuilding or all keeping the
// cells (the parity is not advanced here)
static hipError_t enqueue_steps(sdem_ctx* X, int k, bool rebuild, hipEvent_t* ev = nullptr) {
  for (int i = 0; i < k; ++i) {
    const int a = (X->cur + i) & 1;
    hipError_t e = launch_step(X->c, X->st[a], X->st[a ^ 1], X->st[2], X->ct[a], X->ct[a ^ 1],
                               X->cfg.precision, rebuild ? 1 : 0, X->stream, ev);
    if (e) return e;
  }
  return hipSuccess;
}

// Whether the next steps that keep the cells run as one eight-step graph.
static bool eight_kept_steps(const sdem_ctx* X, int64_t left) {
  return left >= 8 && X->since + 8 <= X->period &&
         (X->n < kDriftCheckEachStep || X->quiet);
}

// Graph patterns: {steps, rebuild}.  A graph bakes in the pointers of both
// buffers for its starting parity.
constexpr int kPatSteps[4] = {2, 1, 1, 8};
constexpr bool kPatRebuild[4] = {true, true, false, false};

static hipGraphExec_t step_graph(sdem_ctx* X, int pat) {
  const int p = X->cur;
  if (X->graph[pat][p] || X->graph_failed || !X->stream) return X->graph[pat][p];
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(X->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    X->graph_failed = true;
    return nullptr;
  }
  hipError_t e = enqueue_steps(X, kPatSteps[pat], kPatRebuild[pat]);
  hipError_t e2 = hipStreamEndCapture(X->stream, &g);
  hipGraphExec_t ex = nullptr;
  if (e || e2 || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    X->graph_failed = true;
    ex = nullptr;
  }
  if (g) (void)hipGraphDestroy(g);
  X->graph[pat][p] = ex;
  if (ex) ++X->graphs_made;
  return ex;
}

// Instantiates, for both buffer parities, every graph pattern that
// sdem_step may launch for this context, so that no capture or
// instantiation happens inside a later run of steps (a timed one, say).
static void prepare_graphs(sdem_ctx* X) {
  if (X->graph_failed || !X->stream) return;
  const int cur = X->cur;
  for (int pat = 0; pat < 4; ++pat) {
    const bool used = !X->c.skin_on ? (pat <= 1) : (pat >= 1);
    if (!used) continue;
    for (int p = 0; p < 2; ++p) {
      X->cur = p;
      (void)step_graph(X, pat);
    }
  }
  X->cur = cur;
}

static hipError_t run_pattern(sdem_ctx* X, int pat) {
  hipGraphExec_t g = step_graph(X, pat);
  hipError_t e = g ? hipGraphLaunch(g, X->stream) : enqueue_steps(X, kPatSteps[pat], kPatRebuild[pat]);
  if (e) return e;
  for (int i = 0; i < kPatSteps[pat]; ++i) count_step(X, kPatRebuild[pat]);
  if (kPatSteps[pat] & 1) X->cur ^= 1;
  return hipSuccess;
}

// At the end of a run of steps since the last rebuild (skin > 0): read the
// drift counters and adapt the period.  A run whose searches had to reach
// past the skin halves the period (down to 4 steps) and forces a rebuild; a
// run without doubles it, up to rebuild_every.
static int adapt_period(sdem_ctx* X, unsigned long long* drift0) {
  Counters h;
  HIP_TRY(hipMemcpyAsync(&h, X->c.ctr, sizeof h, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if (h.flags) return SDEM_OK;  // reported by the caller
  if (h.rebuild_next) X->need_rebuild = true;
  X->quiet = h.drift_steps == *drift0;
  if (!X->quiet)
    X->period = std::max(std::min(4, X->rebuild_every), X->period / 2);
  else
    X->period = std::min(X->rebuild_every, X->period * 2);
  *drift0 = h.drift_steps;
  return SDEM_OK;
}

// The drift flag copied behind the single kept step two steps ago, if any.
static hipError_t lag_take(sdem_ctx* X) {
  const int s = X->lag_slot;
  if (!X->lag_valid[s]) return hipSuccess;
  const hipError_t e = hipEventSynchronize(X->lag_ev[s]);
  if (e) return e;
  if (X->lag_host[s]) X->need_rebuild = true;
  X->lag_valid[s] = false;
  return hipSuccess;
}
// Behind a single kept step of a large context: its drift flag to the host.
static hipError_t lag_put(sdem_ctx* X) {
  const int s = X->lag_slot;
  hipError_t e = hipMemcpyAsync(&X->lag_host[s], &X->c.ctr->rebuild_next, sizeof(int32_t),
                                hipMemcpyDeviceToHost, X->stream);
  if (!e) e = hipEventRecord(X->lag_ev[s], X->stream);
  if (e) return e;
  X->lag_valid[s] = true;
  X->lag_slot ^= 1;
  return hipSuccess;
}
// A rebuild makes the pending flags moot; at the end of a call both are read.
static void lag_drop(sdem_ctx* X) { X->lag_valid[0] = X->lag_valid[1] = false; }
static hipError_t lag_flush(sdem_ctx* X) {
  hipError_t e = lag_take(X);
  X->lag_slot ^= 1;
  if (!e) e = lag_take(X);
  X->lag_slot ^= 1;
  return e;
}
static bool lag_on(const sdem_ctx* X) { return X->lag_host && X->n >= kDriftCheckEachStep; }

int sdem_step(sdem_ctx* X, int64_t nsteps) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->failed) return fail(SDEM_ESTATE, "context failed in an earlier step; read it and re-init");
  if (nsteps < 0) return fail(SDEM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return SDEM_OK;
  X->stepped = true;
  Counters before;
  HIP_TRY(hipMemcpyAsync(&before, X->c.ctr, sizeof before, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  const int start = X->cur;
  unsigned long long drift0 = before.drift_steps;
  int64_t left = nsteps;
  if (!spawning(X)) prepare_graphs(X);
  while (left > 0) {
    if (spawning(X)) {
      // steps one at a time, each after its spawn attempts, without graphs
      // (the particle count may change every step)
      bool stop = false;
      int rc = spawn_now(X, &stop);
      if (rc) return rc;
      if (stop) break;
      if (X->c.skin_on && X->since >= X->period && X->since > 0) {
        rc = adapt_period(X, &drift0);
        if (rc) return rc;
      }
      const bool rb = rebuild_now(X);
      HIP_TRY(enqueue_steps(X, 1, rb));
      count_step(X, rb);
      X->cur ^= 1;
      --left;
      continue;
    }
    int pat;
    if (!X->c.skin_on) {
      pat = left >= 2 ? 0 : 1;
    } else {
      if (lag_on(X)) HIP_TRY(lag_take(X));
      if (X->since >= X->period && X->since > 0) {
        const int rc = adapt_period(X, &drift0);
        if (rc) return rc;
      }
      if (rebuild_now(X))
        pat = 1;
      else if (eight_kept_steps(X, left))
        pat = 3;
      else
        pat = 2;
    }
    HIP_TRY(run_pattern(X, pat));
    left -= kPatSteps[pat];
    if (X->c.skin_on && lag_on(X)) {
      if (kPatRebuild[pat])
        lag_drop(X);
      else if (pat == 2)
        HIP_TRY(lag_put(X));
    }
  }
  if (lag_on(X)) HIP_TRY(lag_flush(X));
  return finish_steps(X, before, start);
}

int sdem_step_profiled(sdem_ctx* X, int64_t nsteps, double* phase_ms) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->failed) return fail(SDEM_ESTATE, "context failed in an earlier step; read it and re-init");
  if (nsteps < 0 || !phase_ms) return fail(SDEM_EINVAL, "bad arguments");
  for (int k = 0; k <= kPhases; ++k) phase_ms[k] = 0.0;
  if (nsteps == 0) return SDEM_OK;
  X->stepped = true;
  hipEvent_t ev[kEvents];
  for (int k = 0; k < kEvents; ++k) HIP_TRY(hipEventCreate(&ev[k]));
  Counters before;
  HIP_TRY(hipMemcpyAsync(&before, X->c.ctr, sizeof before, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  const int start = X->cur;
  unsigned long long drift0 = before.drift_steps;
  hipError_t err = hipSuccess;
  int in_run = 0;  // steps left of what sdem_step would run as one eight-step graph
  for (int64_t i = 0; i < nsteps && !err; ++i) {
    // the same rebuild decisions as sdem_step: the period adapted at its
    // end, eight-step runs where sdem_step would launch them, and large
    // contexts look at the drift flag after each kept step run on its own
    int rc = SDEM_OK;
    if (spawning(X)) {
      bool stop = false;
      rc = spawn_now(X, &stop);
      if (!rc && stop) break;
    }
    const bool lag = X->c.skin_on && lag_on(X) && !spawning(X);
    if (!rc && lag && in_run == 0 && lag_take(X) != hipSuccess)
      rc = fail(SDEM_EHIP, "profiled step failed: %s", hipGetErrorString(hipGetLastError()));
    if (!rc && X->c.skin_on && X->since >= X->period && X->since > 0) rc = adapt_period(X, &drift0);
    if (rc) {
      for (int k = 0; k < kEvents; ++k) (void)hipEventDestroy(ev[k]);
      return rc;
    }
    const bool rb = rebuild_now(X);
    if (in_run == 0 && !rb && X->c.skin_on && !spawning(X) && eight_kept_steps(X, nsteps - i))
      in_run = 8;
    const bool single = in_run == 0;
    if (in_run > 0) --in_run;
    err = enqueue_steps(X, 1, rb, ev);
    count_step(X, rb);
    X->cur ^= 1;
    if (!err && lag) {
      if (rb)
        lag_drop(X);
      else if (single)
        err = lag_put(X);
    }
    if (!err) err = hipEventSynchronize(ev[kPhases]);
    for (int k = 0; k < kPhases && !err; ++k) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      phase_ms[k] += ms;
    }
    if (!err) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[kPhases + 1], ev[kPhases + 2]);
      phase_ms[kPhases] += ms;
    }
  }
  for (int k = 0; k < kEvents; ++k) (void)hipEventDestroy(ev[k]);
  if (!err && lag_on(X)) err = lag_flush(X);
  if (err) return fail(SDEM_EHIP, "profiled step failed: %s", hipGetErrorString(err));
  for (int k = 0; k <= kPhases; ++k) phase_ms[k] /= (double)nsteps;
  return finish_steps(X, before, start);
}

int sdem_read_state(sdem_ctx* X, double* x, double* v, double* w, double* q, double* F,
                    double* T) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  const int64_t n = X->n;
  if (n == 0) return SDEM_OK;
  double* dst[6] = {x, v, w, q, F, T};
  double* dev[6];
  const size_t words[6] = {3, 3, 3, 4, 3, 3};
  size_t at = 0;
  for (int k = 0; k < 6; ++k) {
    if (!dst[k]) {
      dev[k] = nullptr;
    } else if (is_device_ptr(dst[k])) {
      dev[k] = dst[k];
    } else {
      dev[k] = X->scratch + at * n;
    }
    at += words[k];
  }
  HIP_TRY(launch_scatter_state(X->c, X->st[X->cur], dev[0], dev[1], dev[2], dev[3], dev[4], dev[5],
                               X->stream));
  for (int k = 0; k < 6; ++k)
    if (dst[k] && dev[k] != dst[k])
      HIP_TRY(hipMemcpyAsync(dst[k], dev[k], sizeof(double) * words[k] * n, hipMemcpyDeviceToHost,
                             X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

int sdem_read_radii(sdem_ctx* X, double* R) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  const int64_t n = X->n;
  if (n == 0) return SDEM_OK;
  if (!R) return fail(SDEM_EINVAL, "R is NULL");
  double* dev = is_device_ptr(R) ? R : X->scratch;
  HIP_TRY(launch_scatter_radii(X->c, X->st[X->cur], dev, X->stream));
  if (dev != R)
    HIP_TRY(hipMemcpyAsync(R, dev, sizeof(double) * n, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

int sdem_read_contacts(sdem_ctx* X, int64_t cap, int64_t* n_out, int32_t* ki, int32_t* kj,
                       double* us, double* ur, double* ut) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (cap < 0) return fail(SDEM_EINVAL, "cap must be >= 0");
  const int64_t n = X->n;
  const Contacts& C = X->ct[X->cur];
  hipStream_t st = X->stream;
  HIP_TRY(hipStreamSynchronize(st));
  // records of a completed step (or loaded history): [off[s], off[s]+cnt[s])
  int32_t total = 0;
  std::vector<int32_t> cnt((size_t)std::max<int64_t>(n, 1)), off((size_t)std::max<int64_t>(n, 1));
  if (n) {
    HIP_TRY(hipMemcpy(cnt.data(), C.cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(off.data(), C.off, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int64_t s = 0; s < n; ++s) total += cnt[s];
  }
  if (n_out) *n_out = total;
  if (!total) return SDEM_OK;
  const size_t Ctot = (size_t)X->c.ngroups * (size_t)X->c.gcap;
  std::vector<int2> KA(Ctot);
  std::vector<double> SA((size_t)kSpr * Ctot);
  HIP_TRY(hipMemcpy(KA.data(), C.key, sizeof(int2) * Ctot, hipMemcpyDeviceToHost));
  if (X->cfg.precision == SDEM_MIXED) {
    std::vector<float> SF((size_t)kSpr * Ctot);
    HIP_TRY(hipMemcpy(SF.data(), C.spr, sizeof(float) * kSpr * Ctot, hipMemcpyDeviceToHost));
    std::copy(SF.begin(), SF.end(), SA.begin());
  } else {
    HIP_TRY(hipMemcpy(SA.data(), C.spr, sizeof(double) * kSpr * Ctot, hipMemcpyDeviceToHost));
  }
  std::vector<int32_t> K1(total), K2(total);
  std::vector<double> SP((size_t)kSpr * total);
  {
    int32_t w = 0;
    for (int64_t s = 0; s < n; ++s)
      for (int32_t k = 0; k < cnt[s]; ++k, ++w) {
        const size_t e = (size_t)off[s] + k;
        K1[w] = KA[e].x;
        K2[w] = KA[e].y;
        for (int j = 0; j < kSpr; ++j) SP[(size_t)kSpr * w + j] = SA[kSpr * e + j];
      }
  }
  std::vector<int32_t> order(total);
  for (int32_t e = 0; e < total; ++e) order[e] = e;
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return K1[a] < K1[b] || (K1[a] == K1[b] && K2[a] < K2[b]);
  });
  const int64_t m = std::min<int64_t>(cap, total);
  std::vector<int32_t> o1(m), o2(m);
  std::vector<double> ous((size_t)3 * m), our((size_t)3 * m), out((size_t)m);
  for (int64_t r = 0; r < m; ++r) {
    const int32_t e = order[r];
    o1[r] = K1[e];
    o2[r] = K2[e];
    for (int k = 0; k < 3; ++k) {
      ous[3 * r + k] = SP[(size_t)kSpr * e + k];
      our[3 * r + k] = SP[(size_t)kSpr * e + 3 + k];
    }
    out[r] = SP[(size_t)kSpr * e + 6];
  }
  if (m) {
    if (ki) HIP_TRY(hipMemcpy(ki, o1.data(), sizeof(int32_t) * m, hipMemcpyDefault));
    if (kj) HIP_TRY(hipMemcpy(kj, o2.data(), sizeof(int32_t) * m, hipMemcpyDefault));
    if (us) HIP_TRY(hipMemcpy(us, ous.data(), sizeof(double) * 3 * m, hipMemcpyDefault));
    if (ur) HIP_TRY(hipMemcpy(ur, our.data(), sizeof(double) * 3 * m, hipMemcpyDefault));
    if (ut) HIP_TRY(hipMemcpy(ut, out.data(), sizeof(double) * m, hipMemcpyDefault));
  }
  return SDEM_OK;
}

int sdem_graph_stats(sdem_ctx* X, int64_t* instantiated, int32_t* failed) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (instantiated) *instantiated = X->graphs_made;
  if (failed) *failed = X->graph_failed ? 1 : 0;
  return SDEM_OK;
}

int sdem_stats(sdem_ctx* X, int64_t* steps, int64_t* pp, int64_t* pw, int64_t* rebuilds) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  Counters h;
  HIP_TRY(hipMemcpyAsync(&h, X->c.ctr, sizeof h, hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  const int64_t done = (int64_t)h.steps - (h.flags ? 1 : 0);
  int64_t a = 0, b = 0;
  {
    std::vector<unsigned long long> gs((size_t)2 * X->c.ngroups);
    HIP_TRY(hipMemcpy(gs.data(), X->c.gstat, sizeof(unsigned long long) * gs.size(),
                      hipMemcpyDeviceToHost));
    for (int32_t q = 0; q < X->c.ngroups; ++q) {
      a += (int64_t)gs[2 * q];
      b += (int64_t)gs[2 * q + 1];
    }
  }
  if (steps) *steps = done;
  if (pp) *pp = a;
  if (pw) *pw = b;
  if (rebuilds) *rebuilds = (int64_t)h.rebuilds;
  return SDEM_OK;
}

int sdem_set_mesh_motion(sdem_ctx* X, int32_t sim, int32_t ngroups,
                         const sdem_mesh_motion* motions, const int32_t* group_of) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->failed) return fail(SDEM_ESTATE, "context failed in an earlier step; read it and re-init");
  if (sim < 0 || sim >= X->nsims) return fail(SDEM_EINVAL, "sim %d out of range", sim);
  if (ngroups < 1 || ngroups > kMotionMax || !motions)
    return fail(SDEM_EINVAL, "ngroups must be in [1, %d]", kMotionMax);
  std::vector<MeshMotion> table((size_t)ngroups);
  for (int32_t g = 0; g < ngroups; ++g) {
    const sdem_mesh_motion& in = motions[g];
    MeshMotion& o = table[g];
    for (int k = 0; k < 3; ++k) {
      if (!isfinite(in.omega[k]) || !isfinite(in.center[k]) || !isfinite(in.amp[k]))
        return fail(SDEM_EINVAL, "motion %d: omega, center and amp must be finite", g);
      o.omega[k] = in.omega[k];
      o.center[k] = in.center[k];
      o.amp[k] = in.amp[k];
    }
    if (!isfinite(in.freq) || !(in.freq >= 0) || !isfinite(in.phase))
      return fail(SDEM_EINVAL, "motion %d: freq >= 0 and phase must be finite", g);
    o.freq = in.freq;
    o.phase = in.phase;
    o.moving = 0;
    for (int k = 0; k < 3; ++k)
      if (o.omega[k] != 0.0 || (o.amp[k] != 0.0 && o.freq != 0.0)) o.moving = 1;
  }
  const size_t nel = X->mesh_r[sim].size();
  std::vector<int32_t> grp(nel, 0);
  for (size_t m = 0; group_of && m < nel; ++m) {
    if (group_of[m] < 0 || group_of[m] >= ngroups)
      return fail(SDEM_EINVAL, "element %zu: motion group %d out of range", m, group_of[m]);
    grp[m] = group_of[m];
  }
  X->motion[sim] = std::move(table);
  X->mesh_grp[sim] = std::move(grp);
  int rc = upload_mesh(X);  // bins over the swept region, parameters, planes
  if (rc) return rc;
  // the mesh at the current time, with its wall motion
  HIP_TRY(launch_mesh_now(X->c, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

int sdem_set_spawn(sdem_ctx* X, int32_t sim, const sdem_spawn_params* p) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (X->failed) return fail(SDEM_ESTATE, "context failed in an earlier step; read it and re-init");
  if (!p) {
    X->spawn_on = false;
    return SDEM_OK;
  }
  if (X->nsims != 1 || sim != 0)
    return fail(SDEM_EINVAL, "spawning needs a context of one simulation (sim 0)");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(p->smin[k]) || !isfinite(p->smax[k]) || !(p->smax[k] >= p->smin[k]))
      return fail(SDEM_EINVAL, "spawn box: s_min <= s_max, finite, on every axis");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(p->v0[k]) || !isfinite(p->w0[k]))
      return fail(SDEM_EINVAL, "spawn v0 and w0 must be finite");
  if (!(p->R_min > 0) || !(p->R_max >= p->R_min) || !isfinite(p->R_max))
    return fail(SDEM_EINVAL, "spawn radii: 0 < R_min <= R_max");
  if (p->n_spawn < 0 || p->n_spawn > kSpawnMax)
    return fail(SDEM_EINVAL, "n_spawn must be in [0, %d]", kSpawnMax);
  if (p->n_max < 0) return fail(SDEM_EINVAL, "n_max must be >= 0");
  if (p->n_max > X->cfg.n_max)
    return fail(SDEM_ECAPACITY, "spawn n_max = %lld exceeds the context's n_max = %lld",
                (long long)p->n_max, (long long)X->cfg.n_max);
  SpawnParams& S = X->spawn;
  for (int k = 0; k < 3; ++k) {
    S.smin[k] = p->smin[k];
    S.smax[k] = p->smax[k];
    S.v0[k] = p->v0[k];
    S.w0[k] = p->w0[k];
  }
  S.Rmin = p->R_min;
  S.Rmax = p->R_max;
  S.n_spawn = (int32_t)p->n_spawn;
  S.sim = 0;
  S.n_max = p->n_max;
  S.key[0] = (uint32_t)p->seed;
  S.key[1] = (uint32_t)(p->seed >> 32);
  hipStream_t st = X->stream;
  HIP_TRY(hipMemcpyAsync(X->c.spawn, &S, sizeof S, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(&X->c.ctr->spawn_attempts, 0,
                         sizeof(unsigned long long) + sizeof(double) + sizeof(int32_t), st));
  // spawned radii up to R_max set the cell edge and the mesh reach
  if (p->R_max > X->rmax[0]) {
    X->rmax[0] = p->R_max;
    const int rc = X->mesh_r[0].empty() ? upload_params(X) : upload_mesh(X);
    if (rc) return rc;
  }
  if (X->wchunk_host.size() < (size_t)((X->n + kWave - 1) / kWave)) {
    X->wchunk_host.resize((size_t)((X->n + kWave - 1) / kWave));
    for (size_t w = 0; w < X->wchunk_host.size(); ++w) X->wchunk_host[w] = (int32_t)w;
  }
  HIP_TRY(hipStreamSynchronize(st));
  X->spawn_on = true;
  return SDEM_OK;
}

int sdem_set_spawn_status(sdem_ctx* X, uint64_t attempts, double carried) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (!(carried == 0.0 || (carried >= X->spawn.Rmin && carried <= X->spawn.Rmax)) || !X->spawn_on)
    return fail(SDEM_EINVAL, "spawning is off, or the carried radius is outside [R_min, R_max]");
  struct {
    unsigned long long a;
    double r;
  } h{attempts, carried};
  HIP_TRY(hipMemcpyAsync(&X->c.ctr->spawn_attempts, &h, sizeof h, hipMemcpyHostToDevice,
                         X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

int sdem_set_clock(sdem_ctx* X, int64_t steps) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (steps < 0) return fail(SDEM_EINVAL, "steps must be >= 0");
  const unsigned long long s = (unsigned long long)steps;
  HIP_TRY(hipMemcpyAsync(&X->c.ctr->steps, &s, sizeof s, hipMemcpyHostToDevice, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  HIP_TRY(launch_mesh_now(X->c, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  return SDEM_OK;
}

int sdem_spawn_status(sdem_ctx* X, int64_t* n, uint64_t* attempts, double* carried) {
  if (!X) return fail(SDEM_EINVAL, "ctx is NULL");
  if (n) *n = X->n;
  if (attempts || carried) {
    Counters h;
    HIP_TRY(hipMemcpyAsync(&h, X->c.ctr, sizeof h, hipMemcpyDeviceToHost, X->stream));
    HIP_TRY(hipStreamSynchronize(X->stream));
    if (attempts) *attempts = h.spawn_attempts;
    if (carried) *carried = h.spawn_carried;
  }
  return SDEM_OK;
}

int sdem_destroy(sdem_ctx* X) {
  if (!X) return SDEM_OK;
  if (X->stream) (void)hipStreamSynchronize(X->stream);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 4; ++q)
      if (X->graph[q][p]) (void)hipGraphExecDestroy(X->graph[q][p]);
  delete X;
  return SDEM_OK;
}

const char* sdem_last_error(void) { return g_err.c_str(); }

int sdem_selftest_rounding(int64_t n, const double* in, const double* in2, double* out,
                           void* hip_stream) {
  if (n < 0 || (n > 0 && (!in || !in2 || !out))) return fail(SDEM_EINVAL, "bad arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  HIP_TRY(launch_selftest(n, in, in2, out, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SDEM_OK;
}

}  // extern "C"
