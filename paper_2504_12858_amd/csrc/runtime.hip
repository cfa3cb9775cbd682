// Host runtime and C ABI of libgrainenv (see include/grainenv.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "grainenv.h"
#include "internal.h"

using ge::Dev;

namespace {

constexpr size_t ALIGN = 256;
constexpr int64_t MAX_CAP_PARTICLES = 1ll << 28;
constexpr int64_t MAX_SITE_RANGE = 16000;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Geometry {
  int32_t n[3];
  int32_t nb[3];
  uint64_t n_cells;
  uint64_t n_bricks;
  uint64_t slots;
  uint64_t field_nodes;
};

struct Layout {
  size_t A, B, P, spawn, spslot, spawn_cnt, spawn_off, newstop, newstop_cnt, S, PS, S2, PS2, snext, shead, sstart,
      bsinfo, ccnt, cstart, bcnt, binfo, bmeta, dlist, dlist_cnt, dpart, dmask, doff, bown, cown, smask, occ, scan_tmp, ckeys, cbits, clist, dirkeys, gtab, gbox,
      stab, sstate, cand, sgrain, fgrid, gcnt, fcmin, fcoarse, mslots, greach, gsite, gdead, cnt, dig, total;
};

uint64_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Cells along axis a: ceil(L / h), or L / h exactly on a periodic axis.
static double cells_along(const ge_params* p, int a) {
  const double m = (p->hi[a] - p->lo[a]) / p->h;
  return ((p->periodic >> a) & 1) ? std::nearbyint(m) : std::ceil(m);
}

const char* check_params(const ge_params* p) {
  if (!p) return "null params";
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(p->lo[a]) || !std::isfinite(p->hi[a])) return "non-finite box";
    if (!(p->hi[a] > p->lo[a])) return "empty or inverted box";
  }
  if (!(std::isfinite(p->lambda0) && p->lambda0 > 0)) return "lambda0 must be positive";
  if (!(std::isfinite(p->h) && p->h > 0)) return "h must be positive";
  if (!(std::isfinite(p->rc) && p->rc > 0)) return "rc must be positive";
  if (p->rc > p->h) return "rc must not exceed h (27-cell stencil)";
  if (p->rc > p->lambda0) return "rc must not exceed lambda0";
  for (int k = 0; k < 2; ++k)
    if (!std::isfinite(p->a[k]) || !std::isfinite(p->b[k]) || p->a[k] < 0) return "bad kinetics";
  if (!std::isfinite(p->theta)) return "non-finite theta";
  if (p->cap_particles < 6 || p->cap_particles > MAX_CAP_PARTICLES) return "cap_particles out of range";
  if (p->cap_stopped < 1 || p->cap_stopped > (1ll << 31)) return "cap_stopped out of range";
  if (p->cap_grains < 1 || p->cap_grains > (1 << 28) - 2) return "cap_grains out of range";
  if (p->cap_sites < 0) return "cap_sites out of range";
  if (p->cap_claim_bricks < 1 || p->cap_claim_bricks > (1ll << 31)) return "cap_claim_bricks out of range";
  double diag = 0;
  double nb_total = 1;
  for (int a = 0; a < 3; ++a) {
    double L = p->hi[a] - p->lo[a];
    // A grain grows across a periodic face by up to one period.
    const double ext = ((p->periodic >> a) & 1) ? 2.0 * L : L;
    diag += ext * ext;
    double nc = cells_along(p, a);
    if (nc > (1 << 20)) return "too many cells along an axis";
    nb_total *= std::ceil(nc / ge::BRICK);
    if (p->field_n[a] < 0 || p->field_n[a] == 1) return "field_n must be 0 or >= 2";
  }
  if (std::sqrt(diag) / p->lambda0 > MAX_SITE_RANGE) return "box too large for lambda0 (site range)";
  if (nb_total * ge::BRICK_CELLS > 4294967295.0) return "too many cells (2^32)";
  if (p->resort_every < 0) return "resort_every must be >= 0";
  if (p->periodic < 0 || p->periodic > 7) return "periodic must be a mask of axes (0..7)";
  if (p->periodic) {
    if (p->cap_grains > (1 << 26) - 8) return "cap_grains out of range for periodic axes";
    for (int a = 0; a < 3; ++a) {
      if (!((p->periodic >> a) & 1)) continue;
      const double m = (p->hi[a] - p->lo[a]) / p->h;
      if (std::fabs(m - std::nearbyint(m)) > 1e-6 * m || std::nearbyint(m) < 3)
        return "a periodic axis must be a whole number (>= 3) of cells h";
    }
  }
  return nullptr;
}

Geometry geometry(const ge_params* p) {
  Geometry g{};
  g.n_cells = 1;
  g.n_bricks = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = (int32_t)std::max(1.0, cells_along(p, a));
    g.nb[a] = (g.n[a] + ge::BRICK - 1) / ge::BRICK;
    g.n_bricks *= (uint64_t)g.nb[a];
  }
  g.n_cells = g.n_bricks * ge::BRICK_CELLS;  // brick-major, padded to whole bricks
  g.slots = ge::CLAIM_POOL_FACTOR * next_pow2((uint64_t)std::max<int64_t>(p->cap_claim_bricks, 1024));
  g.field_nodes = 1;
  for (int a = 0; a < 3; ++a) g.field_nodes *= (uint64_t)std::max(p->field_n[a], 0);
  if (p->field_n[0] == 0) g.field_nodes = 0;
  return g;
}

Layout layout(const ge_params* p, const Geometry& g) {
  Layout L{};
  size_t off = 0;
  auto put = [&](size_t bytes) {
    size_t o = off;
    off += align_up(std::max<size_t>(bytes, 1));
    return o;
  };
  const uint64_t cp = (uint64_t)p->cap_particles, cs = (uint64_t)p->cap_stopped;
  const uint64_t ntiles = (g.n_bricks + 2047) / 2048;
  L.A = put(16 * cp);
  L.B = put(16 * cp);
  L.P = put(16 * cp);
  L.spawn = put(4 * cp);
  L.spslot = put(4 * cp);
  L.spawn_cnt = put(4 * ge::STREAM_GRID);
  L.spawn_off = put(4 * (ge::STREAM_GRID + 1));
  L.newstop = put(4 * cp);
  L.newstop_cnt = put(4 * ge::STREAM_GRID);
  L.S = put(16 * cs);
  L.PS = put(16 * cs);
  L.S2 = put(16 * cs);
  L.PS2 = put(16 * cs);
  L.snext = put(4 * cs);
  L.shead = put(4 * g.n_cells);
  L.sstart = put(4 * g.n_cells);
  L.bsinfo = put(8 * g.n_bricks);
  L.ccnt = put(4 * g.n_cells);
  L.cstart = put(4 * g.n_cells);
  L.bcnt = put(4 * g.n_bricks);
  L.binfo = put(8 * g.n_bricks);
  L.bmeta = put(16 * g.n_bricks);
  L.dlist = put(4 * g.n_bricks);
  L.dlist_cnt = put(4 * ge::STREAM_GRID);
  L.dpart = put(4 * cp);
  L.bown = put(8 * g.n_bricks);
  L.dmask = put(8 * g.n_bricks);
  L.doff = put(4 * g.n_bricks);
  L.cown = put(8 * g.n_cells);
  L.smask = put(4 * g.n_cells);
  L.occ = put(4 * g.n_bricks);
  L.scan_tmp = put(8 * ntiles);
  L.ckeys = put(8 * g.slots);
  L.cbits = put(192 * g.slots);
  L.clist = put(8 * g.slots);
  L.dirkeys = put(8 * (g.slots / ge::CLAIM_BLOCK_SLOTS));
  L.gtab = put(4 * ge::GT_STRIDE * (uint64_t)p->cap_grains);
  L.gbox = put(24 * (uint64_t)p->cap_grains);
  L.stab = put(4 * ge::GT_STRIDE * (uint64_t)std::max(p->cap_sites, 1));
  L.sstate = put(4 * (uint64_t)std::max(p->cap_sites, 1));
  L.cand = put(4 * (uint64_t)std::max(p->cap_sites, 1));
  L.sgrain = put(4 * (uint64_t)std::max(p->cap_sites, 1));
  L.fgrid = put(4 * std::max<uint64_t>(g.field_nodes, 8));
  L.gcnt = put(4 * std::max<uint64_t>(g.field_nodes, 8));
  L.fcmin = put(4 * std::max<uint64_t>(g.field_nodes, 8));
  // ceil((n - 1) / 4) <= n / 2 for every n >= 2 nodes per axis, so the
  // coarse cells number at most a eighth of the nodes.
  L.fcoarse = put(4 * std::max<uint64_t>(g.field_nodes / 8 + 1, 8));
  L.mslots = put(4 * g.slots);
  L.greach = put(4 * (uint64_t)p->cap_grains);
  L.gsite = put(4 * (uint64_t)p->cap_grains);
  L.gdead = put(4 * (uint64_t)p->cap_grains);
  L.cnt = put(sizeof(ge::Counters));
  L.dig = put(64);
  L.total = off;
  return L;
}

// Grain-table row from centre and quaternion (FP64 maths, FP32 storage).
void grain_row(const double c[3], const double q_in[4], double lambda0, float* row) {
  double w = q_in[0], x = q_in[1], y = q_in[2], z = q_in[3];
  double nq = std::sqrt(w * w + x * x + y * y + z * z);
  w /= nq; x /= nq; y /= nq; z /= nq;
  double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                 2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                 2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  std::memset(row, 0, sizeof(float) * ge::GT_STRIDE);
  for (int a = 0; a < 3; ++a) row[a] = (float)c[a];
  for (int k = 0; k < 9; ++k) {
    row[4 + k] = (float)R[k];
    row[13 + k] = (float)(lambda0 * R[k]);
  }
}

uint4 host_rec(float s, uint32_t g, int d, int sx, int sy, int sz, uint32_t fl) {
  uint4 r;
  std::memcpy(&r.x, &s, 4);
  r.y = (g << 3) | (uint32_t)d;
  r.z = ((uint32_t)(uint16_t)sx) | ((uint32_t)(uint16_t)sy << 16);
  r.w = ((uint32_t)(uint16_t)sz) | (fl << 16);
  return r;
}

}  // namespace

struct ge_ctx {
  ge_params p;
  Geometry geo;
  Layout lay;
  hipStream_t stream;
  char* ws;
  Dev d;
  ge::Counters* host_cnt;  // pinned
  uint32_t* host_word;     // pinned: record count of the allocation-free query
  void* noalloc = nullptr; // this device's scratch of the allocation-free query
  ge_field field;
  std::vector<float> grid_copy;
  int32_t resort_every;
  uint32_t n_sites;
  uint64_t dev_version = 0;  // bumped whenever the launch arguments change
  uint64_t hstep = 0;        // steps taken (host mirror of the device count)
  // recorded step sequence: resort_every steps starting at a multiple of
  // resort_every, replayed with one hipGraphLaunch
  bool use_graphs = true;
  bool graph_valid = false;
  hipGraphExec_t gexec = nullptr;
  uint64_t gversion = 0;
  double gdt = 0.0;
  hipStream_t cap_stream = nullptr;  // capture stream (the context's stream may be the null stream)
  // mushy-zone deposition grid (nodes 0: off) and the volume of its cells
  uint64_t dep_nodes = 0;
  double dep_cell_volume = 0.0;
  std::vector<double> site_xyz;  // registered nucleation sites (grain-to-site link of loaded states)
  // FP64 definitions kept for saved states: the nucleation sites (threshold
  // and quaternion beside site_xyz) and the grains defined on the host
  // (ge_init_grains, loaded states), by grain id; nucleated grains take
  // their site's.
  std::vector<double> site_dT64, site_q64;
  std::vector<double> grain_c64, grain_q64;
  std::vector<uint8_t> grain_host;
  bool dead;
  std::string err;
  // phase timing
  bool prof_on = false;
  bool capturing = false;            // a step sequence is being recorded
  int prof_one = -1;                 // phase timed alone (ge_profile_phase), -1: none
  std::vector<hipEvent_t> ev_pool;   // GE_N_PHASES + 1 (or 2) events per recorded step
  size_t ev_used = 0;                // events recorded since the last read
  double prof_ms[GE_N_PHASES] = {0};
  int64_t prof_steps = 0;
  // adjoint: the caller's workspace of the last recorded run
  struct Adj {
    bool valid = false;
    char* ws = nullptr;
    uint32_t n = 0;
    int32_t n_steps = 0, K = 0;
    float dt = 0.0f;
    size_t tagA, tagB, rec, nact, sfin, ck, seg, xN, dldx, linc, part, grad, mis, total;
  } adj;
};

static const char* PHASE_NAMES[GE_N_PHASES] = {
    "resample", "advance",  "branch",   "scan",   "scatter", "children",
    "dirty",    "contain", "stoplink", "nucleate", "finish", "resort"};

// The next event of the pool (null if none can be created).
static hipEvent_t pool_event(ge_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Records the event that closes phase `k` of the current step (k = -1 opens
// the step).  The single-phase timer records only the two events around its
// phase.  Neither records while a step sequence is being recorded.
static void prof_mark(ge_ctx* c, int k) {
  if (c->capturing) return;
  if (c->prof_one >= 0) {
    if (k != c->prof_one - 1 && k != c->prof_one) return;
    const hipEvent_t e = pool_event(c);
    if (e) (void)hipEventRecord(e, c->stream);
    return;
  }
  if (!c->prof_on) return;
  const hipEvent_t e = pool_event(c);
  if (!e) {
    c->prof_on = false;
    return;
  }
  (void)hipEventRecord(e, c->stream);
}

static void prof_collect(ge_ctx* c) {
  if (c->ev_used == 0) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->prof_one >= 0) {
    const size_t steps = c->ev_used / 2;
    for (size_t st = 0; st < steps; ++st) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, c->ev_pool[2 * st], c->ev_pool[2 * st + 1]) == hipSuccess)
        c->prof_ms[c->prof_one] += ms;
    }
    c->prof_steps += (int64_t)steps;
    c->ev_used = 0;
    return;
  }
  const size_t per = GE_N_PHASES + 1;
  const size_t steps = c->ev_used / per;
  for (size_t st = 0; st < steps; ++st)
    for (int k = 0; k < GE_N_PHASES; ++k) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, c->ev_pool[st * per + k], c->ev_pool[st * per + k + 1]) ==
          hipSuccess)
        c->prof_ms[k] += ms;
    }
  c->prof_steps += (int64_t)steps;
  c->ev_used = 0;
}

static ge_status fail(ge_ctx* c, ge_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

static ge_status hip_check(ge_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return GE_OK;
  if (c) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    c->dead = true;
  }
  return GE_EDEVICE;
}

#define HIPCHK(c, call)                                         \
  do {                                                          \
    ge_status _s = hip_check((c), (call), #call);               \
    if (_s != GE_OK) return _s;                                 \
  } while (0)

static ge_status read_counters(ge_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->host_cnt, c->d.cnt, sizeof(ge::Counters), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

static ge_status write_counters(ge_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->d.cnt, c->host_cnt, sizeof(ge::Counters), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

static ge_status error_status(ge_ctx* c, uint32_t err) {
  err &= ~ge::HOLD;  // a held context is not in error
  if (err == 0) return GE_OK;
  c->dead = true;
  if (err & ge::ERR_CAPACITY) return fail(c, GE_ECAPACITY, "capacity exceeded on the device");
  if (err & ge::ERR_NUMERIC) return fail(c, GE_ENUMERIC, "non-finite undercooling or travel");
  return fail(c, GE_ECFL, "CFL violated: v dt > rc/2 or travel >= 2 lambda0");
}

// Resets the device state (cell lists, claims, counters) to empty.
static ge_status reset_device(ge_ctx* c) {
  const Layout& L = c->lay;
  const Geometry& g = c->geo;
  hipStream_t s = c->stream;
  char* w = c->ws;
  HIPCHK(c, hipMemsetAsync(w + L.shead, 0xFF, 4 * g.n_cells, s));
  HIPCHK(c, hipMemsetAsync(w + L.ccnt, 0, 4 * g.n_cells, s));
  HIPCHK(c, hipMemsetAsync(w + L.bcnt, 0, 4 * g.n_bricks, s));
  HIPCHK(c, hipMemsetAsync(w + L.dlist_cnt, 0, 4 * ge::STREAM_GRID, s));
  HIPCHK(c, hipMemsetAsync(w + L.bown, 0, 8 * g.n_bricks, s));
  HIPCHK(c, hipMemsetAsync(w + L.cown, 0xFF, 8 * g.n_cells, s));
  HIPCHK(c, hipMemsetAsync(w + L.smask, 0, 4 * g.n_cells, s));
  HIPCHK(c, hipMemsetAsync(w + L.bsinfo, 0, 8 * g.n_bricks, s));
  HIPCHK(c, hipMemsetAsync(w + L.spawn_cnt, 0, 4 * ge::STREAM_GRID, s));
  HIPCHK(c, hipMemsetAsync(w + L.newstop_cnt, 0, 4 * ge::STREAM_GRID, s));
  HIPCHK(c, hipMemsetAsync(w + L.ckeys, 0xFF, 8 * g.slots, s));
  HIPCHK(c, hipMemsetAsync(w + L.dirkeys, 0xFF, 8 * (g.slots / ge::CLAIM_BLOCK_SLOTS), s));
  HIPCHK(c, hipMemsetAsync(w + L.cbits, 0, 192 * g.slots, s));
  HIPCHK(c, hipMemsetAsync(w + L.cnt, 0, sizeof(ge::Counters), s));
  HIPCHK(c, hipMemsetAsync(w + L.cand, 0, 4 * (uint64_t)std::max(c->p.cap_sites, 1), s));
  HIPCHK(c, hipMemsetAsync(w + L.sgrain, 0xFF, 4 * (uint64_t)std::max(c->p.cap_sites, 1), s));
  HIPCHK(c, hipMemsetAsync(w + L.greach, 0, 4 * (uint64_t)c->p.cap_grains, s));
  HIPCHK(c, hipMemsetAsync(w + L.gsite, 0xFF, 4 * (uint64_t)c->p.cap_grains, s));
  HIPCHK(c, hipMemsetAsync(w + L.gdead, 0, 4 * (uint64_t)c->p.cap_grains, s));
  ge::launch_init_workspace(c->d, s);  // brick summaries; the step stamps start at 1
  HIPCHK(c, hipGetLastError());
  return GE_OK;
}

// The launch arguments changed (schedule, model, field, sites, adjoint
// recording): recorded step sequences must be recorded again.
static ge_status sync_dev(ge_ctx* c) {
  c->dev_version += 1;
  return GE_OK;
}

static void step_once(ge_ctx* c, double dt);
static ge_status sync_dev(ge_ctx* c);
static ge_status ensure_graph(ge_ctx* c, double dt);

extern "C" {

ge_status ge_validate_params(const ge_params* p) { return check_params(p) ? GE_EINVAL : GE_OK; }

ge_status ge_workspace_size(const ge_params* p, size_t* bytes) {
  if (!bytes || check_params(p)) return GE_EINVAL;
  Geometry g = geometry(p);
  *bytes = layout(p, g).total;
  return GE_OK;
}

// Why the last ge_create on this thread failed (ge_last_error(NULL)).
static thread_local std::string g_create_err;

ge_status ge_create(const ge_params* p, void* workspace, size_t bytes, void* stream,
                    ge_ctx** out) {
  g_create_err.clear();
  if (!out || !workspace) return GE_EINVAL;
  *out = nullptr;
  if (check_params(p)) return GE_EINVAL;
  if (((uintptr_t)workspace) % ALIGN) return GE_EINVAL;
  ge_ctx* c = new ge_ctx();
  c->p = *p;
  c->geo = geometry(p);
  c->lay = layout(p, c->geo);
  if (bytes < c->lay.total) {
    delete c;
    return GE_EINVAL;
  }
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->resort_every = p->resort_every > 0 ? p->resort_every : 16;
  c->n_sites = 0;
  c->dead = false;
  c->field = ge_field{};
  c->field.kind = GE_FIELD_UNIFORM;
  if (hipHostMalloc((void**)&c->host_cnt, sizeof(ge::Counters), hipHostMallocDefault) !=
      hipSuccess) {
    g_create_err = "pinned counters: " + std::string(hipGetErrorString(hipGetLastError()));
    delete c;
    return GE_EDEVICE;
  }
  std::memset(c->host_cnt, 0, sizeof(ge::Counters));
  if (hipHostMalloc((void**)&c->host_word, 64, hipHostMallocDefault) != hipSuccess) {
    g_create_err = "pinned word: " + std::string(hipGetErrorString(hipGetLastError()));
    (void)hipHostFree(c->host_cnt);
    delete c;
    return GE_EDEVICE;
  }
  // The static scratch of the allocation-free query, on the current device.
  if (const hipError_t e = ge::noalloc_scratch(&c->noalloc); e != hipSuccess) {
    g_create_err = "static scratch: " + std::string(hipGetErrorString(e));
    (void)hipGetLastError();
    (void)hipHostFree(c->host_word);
    (void)hipHostFree(c->host_cnt);
    delete c;
    return GE_EDEVICE;
  }
  const Layout& L = c->lay;
  const Geometry& g = c->geo;
  char* w = c->ws;
  Dev& d = c->d;
  std::memset(&d, 0, sizeof(Dev));
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = (float)p->lo[a];
    d.hi[a] = (float)p->hi[a];
    d.n[a] = g.n[a];
    d.nb[a] = g.nb[a];
  }
  d.inv_h = (float)(1.0 / p->h);
  d.n_bricks = (uint32_t)g.n_bricks;
  d.stencil8 = (2.0 * p->rc <= p->h) ? 1 : 0;
  d.periodic = p->periodic;
  for (int a = 0; a < 3; ++a) {
    const double L = p->hi[a] - p->lo[a];
    d.L[a] = (float)L;
    d.invL[a] = (float)(1.0 / L);
  }
  d.lambda0 = (float)p->lambda0;
  d.rc2 = (float)(p->rc * p->rc);
  d.rc_half = (float)(0.5 * p->rc);
  d.ka[0] = (float)p->a[0];
  d.ka[1] = (float)p->a[1];
  d.kb[0] = (float)p->b[0];
  d.kb[1] = (float)p->b[1];
  d.kin_poly = (p->b[0] == 2.0 && p->b[1] == 3.0) ? 1 : 0;
  d.theta = (float)p->theta;
  d.branching = p->branching;
  d.box_exit = p->box_exit;
  d.fkind = ge::F_UNIFORM;
  d.fdT = 0.0f;
  d.fgrid = (float*)(w + L.fgrid);
  d.fcmin = (float*)(w + L.fcmin);
  d.fcoarse = (float*)(w + L.fcoarse);
  d.mslots = (uint32_t*)(w + L.mslots);
  d.greach = (uint32_t*)(w + L.greach);
  d.gsite = (int32_t*)(w + L.gsite);
  d.gdead = (uint32_t*)(w + L.gdead);
  d.gtab = (float*)(w + L.gtab);
  d.gbox = (int32_t*)(w + L.gbox);
  d.cap_grains = (uint32_t)p->cap_grains;
  d.A = (uint4*)(w + L.A);
  d.B = (uint4*)(w + L.B);
  d.P = (float4*)(w + L.P);
  d.cap_p = (uint32_t)p->cap_particles;
  d.spawn = (uint32_t*)(w + L.spawn);
  d.spslot = (uint32_t*)(w + L.spslot);
  d.spawn_cnt = (uint32_t*)(w + L.spawn_cnt);
  d.spawn_off = (uint32_t*)(w + L.spawn_off);
  d.newstop = (uint32_t*)(w + L.newstop);
  d.newstop_cnt = (uint32_t*)(w + L.newstop_cnt);
  d.S = (uint4*)(w + L.S);
  d.PS = (float4*)(w + L.PS);
  d.S2 = (uint4*)(w + L.S2);
  d.PS2 = (float4*)(w + L.PS2);
  d.snext = (uint32_t*)(w + L.snext);
  d.cap_s = (uint32_t)std::min<int64_t>(p->cap_stopped, 0xFFFFFFFEll);
  d.shead = (uint32_t*)(w + L.shead);
  d.sstart = (uint32_t*)(w + L.sstart);
  d.bsinfo = (uint2*)(w + L.bsinfo);
  d.ccnt = (uint32_t*)(w + L.ccnt);
  d.cstart = (uint32_t*)(w + L.cstart);
  d.bcnt = (uint32_t*)(w + L.bcnt);
  d.binfo = (uint2*)(w + L.binfo);
  d.bmeta = (uint4*)(w + L.bmeta);
  d.dlist = (uint32_t*)(w + L.dlist);
  d.dlist_cnt = (uint32_t*)(w + L.dlist_cnt);
  d.dpart = (uint32_t*)(w + L.dpart);
  d.bown = (uint2*)(w + L.bown);
  d.dmask = (unsigned long long*)(w + L.dmask);
  d.doff = (uint32_t*)(w + L.doff);
  d.cown = (uint2*)(w + L.cown);
  d.smask = (uint32_t*)(w + L.smask);
  d.occ = (uint32_t*)(w + L.occ);
  d.scan_tmp = (uint64_t*)(w + L.scan_tmp);
  d.ckeys = (unsigned long long*)(w + L.ckeys);
  d.clist = (unsigned long long*)(w + L.clist);
  d.cbits = (unsigned long long*)(w + L.cbits);
  d.dirkeys = (unsigned long long*)(w + L.dirkeys);
  d.cmask = g.slots - 1;
  d.dirmask = g.slots / ge::CLAIM_BLOCK_SLOTS - 1;
  d.claim_limit = (uint32_t)std::min<uint64_t>(g.slots, 0xFFFFFFFFull);
  const uint64_t blocks = g.slots / ge::CLAIM_BLOCK_SLOTS;
  d.dir_limit = (uint32_t)std::min<uint64_t>(blocks - blocks / 4, 0xFFFFFFFFull);
  d.stab = (float*)(w + L.stab);
  d.sstate = (uint32_t*)(w + L.sstate);
  d.cand = (uint32_t*)(w + L.cand);
  d.sgrain = (uint32_t*)(w + L.sgrain);
  d.n_sites = 0;
  d.cnt = (ge::Counters*)(w + L.cnt);
  d.resort_every = c->resort_every;
  ge_status st = hip_check(c, ge::resident_grids(d), "occupancy query");
  if (st == GE_OK) st = sync_dev(c);
  if (st == GE_OK) st = reset_device(c);
  if (st == GE_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "create");
  if (st != GE_OK) {
    g_create_err = c->err;
    (void)hipHostFree(c->host_cnt);
    (void)hipHostFree(c->host_word);
    delete c;
    return st;
  }
  *out = c;
  return GE_OK;
}

ge_status ge_destroy(ge_ctx* c) {
  if (!c) return GE_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  (void)hipHostFree(c->host_cnt);
  (void)hipHostFree(c->host_word);
  delete c;
  return GE_OK;
}

const char* ge_last_error(const ge_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

// Keeps the FP64 centre and quaternion of grains g0 .. g0 + n - 1 defined on
// the host (for saved states).
static void remember_grains(ge_ctx* c, uint32_t g0, int32_t n, const double* centre,
                            const double* quat) {
  const size_t end = (size_t)g0 + (size_t)n;
  if (c->grain_host.size() < end) {
    c->grain_host.resize(end, 0);
    c->grain_c64.resize(3 * end, 0.0);
    c->grain_q64.resize(4 * end, 0.0);
  }
  for (int32_t i = 0; i < n; ++i) {
    const size_t g = (size_t)g0 + (size_t)i;
    c->grain_host[g] = 1;
    std::memcpy(&c->grain_c64[3 * g], centre + 3 * i, 3 * sizeof(double));
    std::memcpy(&c->grain_q64[4 * g], quat + 4 * i, 4 * sizeof(double));
  }
}

ge_status ge_init_grains(ge_ctx* c, int32_t n, const double* centre, const double* quat,
                         const int32_t* shell_r, uint32_t* first_id) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (n < 0 || (n > 0 && (!centre || !quat || !shell_r))) return fail(c, GE_EINVAL, "bad arguments");
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  ge::Counters& H = *c->host_cnt;
  if (H.err) return error_status(c, H.err);
  const uint32_t g0 = H.n_grains;
  if ((int64_t)g0 + n > c->p.cap_grains) return fail(c, GE_ECAPACITY, "cap_grains exceeded");
  std::vector<float> rows((size_t)n * ge::GT_STRIDE);
  std::vector<int32_t> boxes((size_t)n * 6);
  std::vector<uint4> recs;
  for (int32_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(centre[3 * i + a])) return fail(c, GE_EINVAL, "non-finite centre");
    const int32_t r = shell_r[i];
    if (r < 0 || r > MAX_SITE_RANGE) return fail(c, GE_EINVAL, "shell_r out of range");
    grain_row(centre + 3 * i, quat + 4 * i, c->p.lambda0, rows.data() + (size_t)i * ge::GT_STRIDE);
    for (int a = 0; a < 3; ++a) {
      boxes[6 * i + a] = -r;
      boxes[6 * i + 3 + a] = r;
    }
    const uint32_t g = g0 + (uint32_t)i;
    if (r == 0) {
      for (int d = 0; d < 6; ++d) recs.push_back(host_rec(0.0f, g, d, 0, 0, 0, ge::ST_ACTIVE));
    } else {
      for (int x = -r; x <= r; ++x)
        for (int y = -(r - std::abs(x)); y <= r - std::abs(x); ++y) {
          const int rz = r - std::abs(x) - std::abs(y);
          const int zs[2] = {-rz, rz};
          for (int k = 0; k < (rz == 0 ? 1 : 2); ++k) {
            const int s[3] = {x, y, zs[k]};
            int a = 0;
            for (int b = 1; b < 3; ++b)
              if (std::abs(s[b]) > std::abs(s[a])) a = b;
            const int d = 2 * a + (s[a] < 0 ? 1 : 0);
            recs.push_back(host_rec(0.0f, g, d, s[0], s[1], s[2], ge::ST_ACTIVE));
          }
        }
    }
  }
  const uint32_t na = H.n_active;
  if ((uint64_t)na + recs.size() > (uint64_t)c->p.cap_particles)
    return fail(c, GE_ECAPACITY, "cap_particles exceeded");
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(c->d.gtab + (size_t)g0 * ge::GT_STRIDE, rows.data(),
                           rows.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d.gbox + (size_t)g0 * 6, boxes.data(), boxes.size() * 4,
                           hipMemcpyHostToDevice, s));
  if (!recs.empty())
    HIPCHK(c, hipMemcpyAsync(((H.par & 1u) ? c->d.B : c->d.A) + na, recs.data(),
                             recs.size() * sizeof(uint4), hipMemcpyHostToDevice, s));
  H.n_grains = g0 + (uint32_t)n;
  H.n_active = na + (uint32_t)recs.size();
  H.n_live += (uint32_t)recs.size();
  st = write_counters(c);
  if (st != GE_OK) return st;
  ge::launch_classify_new(c->d, na, (uint32_t)recs.size(), true, s);
  for (int32_t i = 0; i < n; ++i) {
    if (shell_r[i] == 0) ge::launch_claim_ball(c->d, g0 + (uint32_t)i, 0, s);
    else ge::launch_claim_ball(c->d, g0 + (uint32_t)i, shell_r[i], s);
  }
  HIPCHK(c, hipGetLastError());
  st = read_counters(c);
  if (st != GE_OK) return st;
  if (c->host_cnt->err) return error_status(c, c->host_cnt->err);
  remember_grains(c, g0, n, centre, quat);
  if (first_id) *first_id = g0;
  return GE_OK;
}

ge_status ge_set_thermal_field(ge_ctx* c, const ge_field* f) {
  if (!c || !f) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  auto fin = [](double v) { return std::isfinite(v); };
  Dev& d = c->d;
  switch (f->kind) {
    case GE_FIELD_UNIFORM:
      if (!fin(f->dT)) return fail(c, GE_ENUMERIC, "non-finite field");
      break;
    case GE_FIELD_LINEAR:
      if (!fin(f->dT0) || !fin(f->rate) || !fin(f->grad[0]) || !fin(f->grad[1]) || !fin(f->grad[2]))
        return fail(c, GE_ENUMERIC, "non-finite field");
      break;
    case GE_FIELD_GRID:
    case GE_FIELD_SOLUTE:
    case GE_FIELD_ROSENTHAL: {
      uint64_t nodes = 1;
      for (int a = 0; a < 3; ++a) {
        if (f->n[a] < 2 || f->n[a] > c->p.field_n[a]) return fail(c, GE_EINVAL, "grid larger than field_n");
        if (!fin(f->origin[a]) || !(f->spacing[a] > 0) || !fin(f->spacing[a]))
          return fail(c, GE_EINVAL, "bad grid geometry");
        nodes *= (uint64_t)f->n[a];
      }
      if (f->kind == GE_FIELD_GRID) {
        if (!f->data) return fail(c, GE_EINVAL, "GRID needs data");
        HIPCHK(c, hipMemcpyAsync(d.fgrid, f->data, nodes * 4,
                                 f->data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 c->stream));
        if (!f->data_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
      } else if (f->kind == GE_FIELD_SOLUTE) {
        if (!f->T || !f->w) return fail(c, GE_EINVAL, "SOLUTE needs T and w");
        if (!fin(f->liq_T) || !fin(f->liq_m)) return fail(c, GE_ENUMERIC, "non-finite liquidus");
        if (f->data_on_device) {
          ge::launch_solute_nodes(f->T, f->w, f->liq_T, f->liq_m, nodes, d.fgrid, c->stream);
          HIPCHK(c, hipGetLastError());
        } else {
          // Node undercooling in FP64, stored in FP32.
          std::vector<float> u(nodes);
          for (uint64_t k = 0; k < nodes; ++k) {
            const double v = (f->liq_T + f->liq_m * f->w[k]) - f->T[k];
            if (!fin(v)) return fail(c, GE_ENUMERIC, "non-finite node value");
            u[k] = (float)v;
          }
          HIPCHK(c, hipMemcpyAsync(d.fgrid, u.data(), nodes * 4, hipMemcpyHostToDevice, c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
        }
      } else {
        const double v[] = {f->dT0, f->rate, f->q, f->U, f->alpha, f->x_start, f->x_end, f->ys,
                            f->zs, f->r_min, f->dT_min, f->grad[0], f->grad[1], f->grad[2]};
        for (double x : v)
          if (!fin(x)) return fail(c, GE_ENUMERIC, "non-finite field");
        if (!(f->alpha > 0) || !(f->x_end > f->x_start)) return fail(c, GE_EINVAL, "bad source");
      }
      break;
    }
    default:
      return fail(c, GE_EINVAL, "unknown field kind");
  }
  c->field = *f;
  c->field.data = nullptr;
  c->field.T = c->field.w = nullptr;
  const Dev before = d;
  // The device interpolates a SOLUTE field's node undercooling like a GRID.
  d.fkind = f->kind == GE_FIELD_SOLUTE ? GE_FIELD_GRID : f->kind;
  d.fdT = (float)f->dT;
  for (int a = 0; a < 3; ++a) {
    d.fgrad[a] = (float)f->grad[a];
    d.fn[a] = f->n[a];
    d.fo[a] = (float)f->origin[a];
    d.finv[a] = f->spacing[a] > 0 ? (float)(1.0 / f->spacing[a]) : 0.0f;
  }
  d.fdT0 = f->dT0;
  d.frate = f->rate;
  ge::Rosenthal& r = d.ros;
  r.dT0 = f->dT0;
  r.rate = f->rate;
  r.q = f->q;
  r.U = f->U;
  r.alpha = f->alpha;
  r.x_start = f->x_start;
  r.x_end = f->x_end;
  r.ys = f->ys;
  r.zs = f->zs;
  r.r_min = f->r_min;
  r.dT_min = f->dT_min;
  for (int a = 0; a < 3; ++a) {
    r.grad[a] = f->grad[a];
    r.o[a] = f->origin[a];
    r.sp[a] = f->spacing[a];
  }
  // Launch arguments unchanged (same kind and geometry, new node values):
  // the recorded step sequence stays valid.
  if (std::memcmp(&before, &d, sizeof(Dev)) == 0) return GE_OK;
  return sync_dev(c);
}

ge_status ge_nucleate(ge_ctx* c, int32_t n, const double* xyz, const double* dT_nuc,
                      const double* quat) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (n < 0 || (n > 0 && (!xyz || !dT_nuc || !quat))) return fail(c, GE_EINVAL, "bad arguments");
  if ((int64_t)c->n_sites + n > c->p.cap_sites) return fail(c, GE_ECAPACITY, "cap_sites exceeded");
  if (n == 0) return GE_OK;
  std::vector<float> rows((size_t)n * ge::GT_STRIDE);
  for (int32_t i = 0; i < n; ++i) {
    if (!std::isfinite(dT_nuc[i])) return fail(c, GE_ENUMERIC, "non-finite nucleation undercooling");
    float* row = rows.data() + (size_t)i * ge::GT_STRIDE;
    grain_row(xyz + 3 * i, quat + 4 * i, c->p.lambda0, row);
    row[3] = (float)dT_nuc[i];
  }
  HIPCHK(c, hipMemcpyAsync(c->d.stab + (size_t)c->n_sites * ge::GT_STRIDE, rows.data(),
                           rows.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d.sstate + c->n_sites, 0, 4 * (size_t)n, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->n_sites += (uint32_t)n;
  c->d.n_sites = c->n_sites;
  c->site_xyz.insert(c->site_xyz.end(), xyz, xyz + 3 * (size_t)n);
  c->site_dT64.insert(c->site_dT64.end(), dT_nuc, dT_nuc + (size_t)n);
  c->site_q64.insert(c->site_q64.end(), quat, quat + 4 * (size_t)n);
  ge_status st = sync_dev(c);
  if (st != GE_OK) return st;
  return GE_OK;
}


static void fill_stats(ge_ctx* c, ge_step_stats* st) {
  const ge::Counters& H = *c->host_cnt;
  st->n_active = (int64_t)H.n_live;
  st->n_stopped = (int64_t)H.n_stopped;
  st->n_grains = (int64_t)H.n_grains;
  st->n_claim_bricks = (int64_t)H.claim_used;
  st->advanced = (int64_t)H.advanced;
  st->exited = (int64_t)H.exited;
  st->spawners = (int64_t)H.spawners;
  st->children = (int64_t)H.children;
  st->contained = (int64_t)H.contained;
  st->nucleated = (int64_t)H.nucleated;
  float ms;
  std::memcpy(&ms, &H.max_step, 4);
  st->max_step = ms;
  st->t = H.t;
  st->step = (int64_t)H.step;
  st->pair_tests = (int64_t)H.pair_tests;
  st->dirty_tests = (int64_t)H.dirty_tests;
  st->melted = (int64_t)H.melted;
  st->removed = (int64_t)H.removed;
  st->reactivated = (int64_t)H.reactivated;
  st->grains_melted = (int64_t)H.grains_melted;
}

ge_status ge_step(ge_ctx* c, double dt, int32_t n_steps, ge_step_stats* stats) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (!(std::isfinite(dt) && dt > 0) || n_steps < 0) return fail(c, GE_EINVAL, "bad dt or n_steps");
  ge::launch_reset_stats(c->d, c->stream);
  int32_t k = 0;
  const int32_t R = c->resort_every;
  if (c->use_graphs && !c->prof_on && c->prof_one < 0 && n_steps >= 2 * R) {
    // Plain steps up to a multiple of resort_every, then whole recorded
    // sequences of resort_every steps, then the rest plain.
    while (k < n_steps && c->hstep % (uint64_t)R != 0) {
      step_once(c, dt);
      ++k;
    }
    const int32_t reps = (n_steps - k) / R;
    if (reps > 0) {
      ge_status st = ensure_graph(c, dt);
      if (st != GE_OK) return st;
      for (int32_t r = 0; r < reps; ++r) HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      k += reps * R;
      c->hstep += (uint64_t)reps * (uint64_t)R;
    }
  }
  for (; k < n_steps; ++k) step_once(c, dt);
  HIPCHK(c, hipGetLastError());
  if (!stats) return GE_OK;
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  fill_stats(c, stats);
  return error_status(c, c->host_cnt->err);
}

}  // extern "C"

// One step of the method on the context's stream (no synchronisation).
// lin_c_out (nullable) receives the LINEAR field's constant of the step.
static void step_once(ge_ctx* c, double dt) {
  hipStream_t s = c->stream;
  const Dev& d = c->d;
  if ((c->prof_on || c->prof_one >= 0) && !c->capturing && c->ev_used + GE_N_PHASES + 1 > 4096)
    prof_collect(c);
  prof_mark(c, -1);
  if (c->field.kind == GE_FIELD_ROSENTHAL) ge::launch_resample(d, s);
  // Melting uses the field of this step.
  if (d.melting) ge::launch_melt(d, s);
  prof_mark(c, 0);
  ge::launch_advance(d, (float)dt, s);
  prof_mark(c, 1);
  ge::launch_branch(d, s);
  prof_mark(c, 2);
  ge::launch_scan(d, s);
  prof_mark(c, 3);
  ge::launch_scatter(d, s);
  prof_mark(c, 4);
  ge::launch_scatter_children(d, s);
  prof_mark(c, 5);
  ge::launch_dirty(d, s);
  prof_mark(c, 6);
  ge::launch_contain(d, s);
  prof_mark(c, 7);
  ge::launch_stoplink(d, s);
  prof_mark(c, 8);
  ge::launch_nucleate(d, s);
  prof_mark(c, 9);
  // Counts the step, advances time, swaps the roles of the active stores.
  ge::launch_finish(d, dt, s);
  prof_mark(c, 10);
  // Re-sort of the stopped store after every resort_every-th step (the
  // kernels check the device step count as well).
  c->hstep += 1;
  if (c->hstep % (uint64_t)c->resort_every == 0) ge::launch_stopped_rebuild(d, s);
  prof_mark(c, 11);
}

// Records resort_every steps from a step count that is a multiple of
// resort_every (nothing runs during the recording) and instantiates them.
static ge_status ensure_graph(ge_ctx* c, double dt) {
  if (c->graph_valid && c->gversion == c->dev_version && c->gdt == dt) return GE_OK;
  if (c->gexec) {
    HIPCHK(c, hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
  }
  c->graph_valid = false;
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const uint64_t h0 = c->hstep;
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    c->capturing = true;
    for (int32_t k = 0; k < c->resort_every; ++k) step_once(c, dt);
    c->capturing = false;
    e = hipStreamEndCapture(c->cap_stream, &g);
  }
  c->stream = user;
  c->hstep = h0;
  HIPCHK(c, e);
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(c, e);
  c->graph_valid = true;
  c->gversion = c->dev_version;
  c->gdt = dt;
  return GE_OK;
}

extern "C" {

// Copies `bytes` of device data at src to out (host or device).
static ge_status deliver(ge_ctx* c, const void* src, void* out, size_t bytes) {
  hipPointerAttribute_t attr;
  bool dev_out = false;
  if (hipPointerGetAttributes(&attr, out) == hipSuccess)
    dev_out = attr.type == hipMemoryTypeDevice;
  (void)hipGetLastError();
  HIPCHK(c, hipMemcpyAsync(out, src, bytes, dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

ge_status ge_query_envelope(ge_ctx* c, int32_t kind, const ge_query_args* args, void* out,
                            size_t out_bytes, size_t* needed) {
  if (!c) return GE_EINVAL;
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  const ge::Counters H = *c->host_cnt;
  hipStream_t s = c->stream;
  size_t need = 0;
  switch (kind) {
    case GE_QUERY_COUNTS: {
      need = sizeof(ge_step_stats);
      if (needed) *needed = need;
      if (!out || out_bytes < need) return GE_OK;
      ge_step_stats v{};
      fill_stats(c, &v);
      v.advanced = v.exited = v.spawners = v.children = v.contained = v.nucleated = 0;
      v.pair_tests = 0;
      v.dirty_tests = 0;
      v.max_step = 0;
      std::memcpy(out, &v, sizeof(v));
      return error_status(c, H.err);
    }
    case GE_QUERY_PARTICLES:
    case GE_QUERY_CLAIMS: {
      const bool parts = kind == GE_QUERY_PARTICLES;
      const size_t rec = parts ? sizeof(ge_particle_rec) : sizeof(ge_claim_rec);
      float winbuf[6];
      const float* win = nullptr;
      if (args) {
        for (int a = 0; a < 3; ++a) {
          winbuf[a] = (float)args->origin[a];
          winbuf[3 + a] = (float)(args->origin[a] + args->n[a] * args->spacing[a]);
        }
        win = winbuf;
      }
      uint32_t* counter = nullptr;
      HIPCHK(c, hipMalloc((void**)&counter, 4));
      HIPCHK(c, hipMemsetAsync(counter, 0, 4, s));
      if (parts) ge::launch_export_particles(c->d, counter, nullptr, 0, win, s);
      else ge::launch_export_claims(c->d, counter, nullptr, 0, win, s);
      uint32_t count = 0;
      HIPCHK(c, hipMemcpyAsync(&count, counter, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      need = (size_t)count * rec;
      if (needed) *needed = need;
      if (!out || out_bytes < need || count == 0) {
        (void)hipFree(counter);
        return GE_OK;
      }
      void* stage = nullptr;
      HIPCHK(c, hipMalloc(&stage, need));
      HIPCHK(c, hipMemsetAsync(counter, 0, 4, s));
      if (parts) ge::launch_export_particles(c->d, counter, stage, count, win, s);
      else ge::launch_export_claims(c->d, counter, stage, count, win, s);
      HIPCHK(c, hipGetLastError());
      st = deliver(c, stage, out, need);
      (void)hipFree(stage);
      (void)hipFree(counter);
      return st;
    }
    case GE_QUERY_GRAIN_MAP: {
      if (!args) return fail(c, GE_EINVAL, "GRAIN_MAP needs args");
      uint64_t nv = 1;
      int32_t n[3];
      float o[3], sp[3];
      for (int a = 0; a < 3; ++a) {
        if (args->n[a] < 1 || !(args->spacing[a] > 0)) return fail(c, GE_EINVAL, "bad voxel grid");
        n[a] = args->n[a];
        o[a] = (float)args->origin[a];
        sp[a] = (float)args->spacing[a];
        nv *= (uint64_t)n[a];
      }
      need = nv * 4;
      if (needed) *needed = need;
      if (!out || out_bytes < need) return GE_OK;
      void* stage = nullptr;
      HIPCHK(c, hipMalloc(&stage, need));
      ge::launch_grain_map(c->d, n, o, sp, (uint32_t*)stage, s);
      HIPCHK(c, hipGetLastError());
      st = deliver(c, stage, out, need);
      (void)hipFree(stage);
      return st;
    }
    case GE_QUERY_SITES: {
      need = (size_t)c->n_sites * 4;
      if (needed) *needed = need;
      if (!out || out_bytes < need || need == 0) return GE_OK;
      return deliver(c, c->d.sstate, out, need);
    }
    case GE_QUERY_DIGEST: {
      need = 3 * sizeof(unsigned long long);
      if (needed) *needed = need;
      if (!out || out_bytes < need) return GE_OK;
      char* dig = c->ws + c->lay.dig;
      HIPCHK(c, hipMemsetAsync(dig, 0, need, c->stream));
      ge::launch_digest(c->d, (unsigned long long*)dig, c->stream);
      HIPCHK(c, hipGetLastError());
      return deliver(c, dig, out, need);
    }
    case GE_QUERY_GRAINS: {
      need = (size_t)H.n_grains * ge::GT_STRIDE * 4;
      if (needed) *needed = need;
      if (!out || out_bytes < need || need == 0) return GE_OK;
      return deliver(c, c->d.gtab, out, need);
    }
    case GE_QUERY_MUSHY_COUNTS:
    case GE_QUERY_MUSHY: {
      if (!c->d.gcnt) return fail(c, GE_EINVAL, "no deposition grid set");
      need = (size_t)c->dep_nodes * 4;
      if (needed) *needed = need;
      if (!out || out_bytes < need) return GE_OK;
      if (kind == GE_QUERY_MUSHY_COUNTS) return deliver(c, c->d.gcnt, out, need);
      // g^m on the device, then to the caller.
      const double site_over_cell =
          (double)c->p.lambda0 * c->p.lambda0 * c->p.lambda0 / c->dep_cell_volume;
      float* tmp = nullptr;
      HIPCHK(c, hipMalloc((void**)&tmp, need));
      ge::launch_mushy_fraction(c->d.gcnt, c->dep_nodes, site_over_cell, tmp, c->stream);
      const ge_status st2 = deliver(c, tmp, out, need);
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(tmp);
      return st2;
    }
    default:
      return fail(c, GE_EINVAL, "unknown query kind");
  }
}

ge_status ge_query_particles_noalloc(ge_ctx* c, const ge_query_args* args, void* out,
                                     size_t out_bytes, size_t* needed) {
  if (!c) return GE_EINVAL;
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  float winbuf[6];
  const float* win = nullptr;
  if (args) {
    for (int a = 0; a < 3; ++a) {
      if (args->n[a] < 1 || !(args->spacing[a] > 0)) return fail(c, GE_EINVAL, "bad window");
      winbuf[a] = (float)args->origin[a];
      winbuf[3 + a] = (float)(args->origin[a] + args->n[a] * args->spacing[a]);
    }
    win = winbuf;
  }
  hipStream_t s = c->stream;
  ge::launch_export_particles_staged(c->d, c->noalloc, win, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->host_word, c->noalloc, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const uint32_t count = *c->host_word;
  const size_t need = (size_t)count * sizeof(ge_particle_rec);
  if (needed) *needed = need;
  if (count > ge::NOALLOC_RECORDS)
    return fail(c, GE_ECAPACITY, "the window holds more particles than the static staging of "
                                 "the allocation-free query (1048576)");
  if (!out || out_bytes < need || count == 0) return GE_OK;
  return deliver(c, (const char*)c->noalloc + ge::NOALLOC_RECORDS_OFFSET, out, need);
}

ge_status ge_profile(ge_ctx* c, int32_t on) {
  if (!c) return GE_EINVAL;
  prof_collect(c);
  c->prof_one = -1;
  if (on) {
    for (double& v : c->prof_ms) v = 0;
    c->prof_steps = 0;
    c->prof_on = true;
  } else {
    c->prof_on = false;
  }
  return GE_OK;
}

ge_status ge_profile_phase(ge_ctx* c, int32_t phase) {
  if (!c) return GE_EINVAL;
  if (phase < -1 || phase >= GE_N_PHASES) return fail(c, GE_EINVAL, "phase out of range");
  prof_collect(c);
  c->prof_on = false;
  c->prof_one = phase;
  for (double& v : c->prof_ms) v = 0;
  c->prof_steps = 0;
  return GE_OK;
}

ge_status ge_profile_read(ge_ctx* c, double* ms, int64_t* steps) {
  if (!c || !ms) return GE_EINVAL;
  prof_collect(c);
  for (int k = 0; k < GE_N_PHASES; ++k) ms[k] = c->prof_ms[k];
  if (steps) *steps = c->prof_steps;
  return GE_OK;
}

const char* ge_phase_name(int32_t k) {
  return (k >= 0 && k < GE_N_PHASES) ? PHASE_NAMES[k] : "";
}

static_assert(GE_N_TUNABLE == ge::TK_N, "tunable kernel count");
static_assert(GE_MAX_BLOCKS == ge::STREAM_GRID, "per-block list capacity");
static const char* TUNABLE_NAMES[GE_N_TUNABLE] = {"advance", "branch", "cellscan", "scatter",
                                                   "children", "dirty", "contain", "stoplink"};
// Phase (profiler index) whose time each tunable kernel dominates.
static const int TUNABLE_PHASE[GE_N_TUNABLE] = {1, 2, 3, 4, 5, 6, 7, 8};

const char* ge_tunable_name(int32_t k) {
  return (k >= 0 && k < GE_N_TUNABLE) ? TUNABLE_NAMES[k] : "";
}

ge_status ge_hold(ge_ctx* c, int32_t on) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  ge::Counters& H = *c->host_cnt;
  H.err = on ? (H.err | ge::HOLD) : (H.err & ~ge::HOLD);
  c->hstep = H.step;
  return write_counters(c);
}

ge_status ge_prepare_step(ge_ctx* c, double dt) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (!(std::isfinite(dt) && dt > 0)) return fail(c, GE_EINVAL, "bad dt");
  return c->use_graphs ? ensure_graph(c, dt) : GE_OK;
}

ge_status ge_use_graphs(ge_ctx* c, int32_t on) {
  if (!c) return GE_EINVAL;
  c->use_graphs = on != 0;
  return GE_OK;
}

ge_status ge_get_schedule(ge_ctx* c, int32_t* blocks) {
  if (!c || !blocks) return GE_EINVAL;
  for (int k = 0; k < GE_N_TUNABLE; ++k) blocks[k] = (int32_t)c->d.sched[k];
  return GE_OK;
}

ge_status ge_set_schedule(ge_ctx* c, const int32_t* blocks) {
  if (!c || !blocks) return GE_EINVAL;
  for (int k = 0; k < GE_N_TUNABLE; ++k)
    if (blocks[k] < 0 || blocks[k] > GE_MAX_BLOCKS) return fail(c, GE_EINVAL, "schedule entry out of range");
  for (int k = 0; k < GE_N_TUNABLE; ++k)
    if (blocks[k] > 0) c->d.sched[k] = (uint32_t)blocks[k];
  return sync_dev(c);
}

ge_status ge_autotune(ge_ctx* c, double dt, int32_t steps_per_trial, void* snapshot,
                      size_t snapshot_bytes, int32_t* blocks_out) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (steps_per_trial < 1) return fail(c, GE_EINVAL, "steps_per_trial must be >= 1");
  if (snapshot && snapshot_bytes < c->lay.total)
    return fail(c, GE_EINVAL, "snapshot smaller than the context's workspace");
  int dev = 0, cus = 0;
  ge_status st = hip_check(c, hipGetDevice(&dev), "autotune");
  if (st == GE_OK)
    st = hip_check(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                   "autotune");
  if (st != GE_OK) return st;
  // Candidates: 1..8 blocks per compute unit, whole multiples of 8 blocks.
  std::vector<uint32_t> cand;
  for (int per = 1; per <= 8; ++per) {
    uint32_t g = (uint32_t)std::min(per * std::max(cus, 1), GE_MAX_BLOCKS);
    g = g >= 8u ? g / 8u * 8u : g;
    if (cand.empty() || cand.back() != g) cand.push_back(g);
  }
  // With a snapshot every trial starts from the state of the call, which is
  // restored at the end.
  const uint64_t hstep0 = c->hstep;
  auto restore = [&]() -> ge_status {
    c->hstep = hstep0;
    return hip_check(c, hipMemcpyAsync(c->ws, snapshot, c->lay.total, hipMemcpyDeviceToDevice,
                                       c->stream), "autotune snapshot");
  };
  if (snapshot &&
      (st = hip_check(c, hipMemcpyAsync(snapshot, c->ws, c->lay.total, hipMemcpyDeviceToDevice,
                                        c->stream), "autotune snapshot")) != GE_OK)
    return st;
  for (int k = 0; k < GE_N_TUNABLE; ++k) {
    uint32_t best = c->d.sched[k];
    double best_cost = INFINITY;
    for (uint32_t g : cand) {
      c->d.sched[k] = g;
      if ((st = sync_dev(c)) != GE_OK) return st;
      if (snapshot && (st = restore()) != GE_OK) return st;
      ge_profile(c, 1);
      ge_step_stats s{};
      st = ge_step(c, dt, steps_per_trial, &s);
      double ms[GE_N_PHASES];
      int64_t steps = 0;
      if (st == GE_OK) st = ge_profile_read(c, ms, &steps);
      ge_profile(c, 0);
      if (st != GE_OK) return st;
      const double cost = ms[TUNABLE_PHASE[k]] / (double)std::max<int64_t>(s.advanced, 1);
      if (cost < best_cost) {
        best_cost = cost;
        best = g;
      }
    }
    c->d.sched[k] = best;
  }
  if ((st = sync_dev(c)) != GE_OK) return st;
  if (snapshot) {
    if ((st = restore()) != GE_OK || (st = read_counters(c)) != GE_OK) return st;
  }
  if (blocks_out) return ge_get_schedule(c, blocks_out);
  return GE_OK;
}

// Loads a state: grains, particles, site states and time from S; the claims
// from S's per-site arrays, or (slots non-null) from n_slots claim-brick
// records of a saved state (host memory).
static ge_status load_state(ge_ctx* c, const ge_state_in& S, const void* slots, int64_t n_slots) {
  if (S.n_grains < 0 || S.n_grains > c->p.cap_grains) return fail(c, GE_ECAPACITY, "cap_grains exceeded");
  if (S.n_particles < 0 || S.n_claims < 0 || n_slots < 0) return fail(c, GE_EINVAL, "negative counts");
  if (n_slots > 0 && (uint64_t)n_slots > c->d.claim_limit)
    return fail(c, GE_ECAPACITY, "cap_claim_bricks too small for the saved claims");
  if ((uint32_t)S.n_sites != c->n_sites) return fail(c, GE_EINVAL, "site count differs from registered sites");
  // Every argument is checked before the device state is touched.
  if ((S.n_grains > 0 && (!S.centre || !S.quat)) ||
      (S.n_particles > 0 && (!S.grain || !S.site || !S.dir || !S.s || !S.state)) ||
      (S.n_claims > 0 && (!S.c_grain || !S.c_site || !S.c_flags)) ||
      (S.n_sites > 0 && !S.site_state))
    return fail(c, GE_EINVAL, "missing arrays");
  int64_t n_keep = 0;
  for (int64_t i = 0; i < S.n_particles; ++i) {
    if (S.state[i] == GE_RETIRED) continue;
    if (S.state[i] != GE_ACTIVE && S.state[i] != GE_STOPPED) return fail(c, GE_EINVAL, "bad particle state");
    if (S.grain[i] < 0 || S.grain[i] >= S.n_grains || S.dir[i] < 0 || S.dir[i] > 5)
      return fail(c, GE_EINVAL, "bad particle");
    // The travel of a live particle stays below 2 lambda0 (the CFL error
    // stops a step before it); kernels rely on that bound.
    if (!(S.s[i] >= 0.0f && S.s[i] < (float)(2.0 * c->p.lambda0)))
      return fail(c, GE_EINVAL, "particle travel outside [0, 2 lambda0)");
    for (int a = 0; a < 3; ++a)
      if (std::abs(S.site[3 * i + a]) > MAX_SITE_RANGE) return fail(c, GE_EINVAL, "site out of range");
    ++n_keep;
  }
  if (n_keep > c->p.cap_particles) return fail(c, GE_ECAPACITY, "cap_particles exceeded");
  for (int64_t k = 0; k < S.n_claims; ++k) {
    if (S.c_grain[k] < 0 || S.c_grain[k] >= S.n_grains) return fail(c, GE_EINVAL, "bad claim grain");
    for (int a = 0; a < 3; ++a)
      if (std::abs(S.c_site[3 * k + a]) > MAX_SITE_RANGE) return fail(c, GE_EINVAL, "claim site out of range");
  }
  hipStream_t s = c->stream;
  c->dead = false;
  c->err.clear();
  ge_status st = reset_device(c);
  if (st != GE_OK) return st;
  // Grains.
  std::vector<float> rows((size_t)S.n_grains * ge::GT_STRIDE);
  std::vector<int32_t> boxes((size_t)S.n_grains * 6);
  for (int32_t g = 0; g < S.n_grains; ++g) {
    grain_row(S.centre + 3 * g, S.quat + 4 * g, c->p.lambda0, rows.data() + (size_t)g * ge::GT_STRIDE);
    for (int a = 0; a < 3; ++a) {
      boxes[6 * g + a] = INT_MAX;
      boxes[6 * g + 3 + a] = INT_MIN;
    }
  }
  // Particles: active and stopped (retired ones are dropped).
  std::vector<uint4> recs;
  recs.reserve((size_t)S.n_particles);
  for (int64_t i = 0; i < S.n_particles; ++i) {
    if (S.state[i] == GE_RETIRED) continue;
    recs.push_back(host_rec(S.s[i], (uint32_t)S.grain[i], S.dir[i], S.site[3 * i], S.site[3 * i + 1],
                            S.site[3 * i + 2],
                            S.state[i] == GE_STOPPED ? ge::ST_STOPPED : ge::ST_ACTIVE));
  }
  // A grain whose centre is the position of a fired site came from that
  // site (it returns to it if it melts entirely).
  std::vector<int32_t> gsite((size_t)S.n_grains, -1);
  for (int32_t g = 0; g < S.n_grains; ++g)
    for (uint32_t i = 0; i < c->n_sites && gsite[g] < 0; ++i)
      if (S.site_state[i] == GE_SITE_FIRED && c->site_xyz[3 * i] == S.centre[3 * g] &&
          c->site_xyz[3 * i + 1] == S.centre[3 * g + 1] && c->site_xyz[3 * i + 2] == S.centre[3 * g + 2])
        gsite[g] = (int32_t)i;
  if (!rows.empty()) {
    HIPCHK(c, hipMemcpyAsync(c->d.gtab, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d.gsite, gsite.data(), gsite.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d.gbox, boxes.data(), boxes.size() * 4, hipMemcpyHostToDevice, s));
  }
  if (!recs.empty())
    HIPCHK(c, hipMemcpyAsync(c->d.A, recs.data(), recs.size() * sizeof(uint4), hipMemcpyHostToDevice, s));
  if (S.n_sites > 0) {
    std::vector<uint32_t> ss(S.site_state, S.site_state + S.n_sites);
    HIPCHK(c, hipMemcpyAsync(c->d.sstate, ss.data(), ss.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  ge::Counters& H = *c->host_cnt;
  std::memset(&H, 0, sizeof(H));
  H.n_grains = (uint32_t)S.n_grains;
  H.n_active = (uint32_t)recs.size();
  H.n_live = (uint32_t)recs.size();
  H.epoch = 1;
  H.t = S.t;
  H.step = (unsigned long long)S.step;
  c->hstep = (uint64_t)S.step;
  st = write_counters(c);
  if (st != GE_OK) return st;
  ge::launch_classify_new(c->d, 0, (uint32_t)recs.size(), false, s);
  if (S.n_claims > 0) {
    const size_t m = (size_t)S.n_claims;
    char* buf = nullptr;
    HIPCHK(c, hipMalloc((void**)&buf, m * 17 + 64));
    int32_t* dg = (int32_t*)buf;
    int32_t* ds = (int32_t*)(buf + m * 4);
    uint8_t* df = (uint8_t*)(buf + m * 16);
    HIPCHK(c, hipMemcpyAsync(dg, S.c_grain, m * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(ds, S.c_site, m * 12, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(df, S.c_flags, m, hipMemcpyHostToDevice, s));
    ge::launch_claim_list(c->d, dg, ds, df, (uint32_t)m, s);
    HIPCHK(c, hipStreamSynchronize(s));
    (void)hipFree(buf);
  }
  if (n_slots > 0) {
    // In chunks of at most 1M claim bricks (144 MB of staging).
    const size_t rec = sizeof(ge_state_claims), chunk = std::min<size_t>((size_t)n_slots, 1u << 20);
    char* buf = nullptr;
    HIPCHK(c, hipMalloc((void**)&buf, chunk * rec));
    for (size_t k = 0; k < (size_t)n_slots; k += chunk) {
      const size_t m = std::min(chunk, (size_t)n_slots - k);
      HIPCHK(c, hipMemcpyAsync(buf, (const char*)slots + k * rec, m * rec, hipMemcpyHostToDevice, s));
      ge::launch_claim_slots(c->d, buf, (uint32_t)m, s);
      HIPCHK(c, hipStreamSynchronize(s));
    }
    (void)hipFree(buf);
  }
  if (c->d.gcnt) {
    // Deposition counts of the loaded claims.
    HIPCHK(c, hipMemsetAsync(c->d.gcnt, 0, 4 * c->dep_nodes, s));
    ge::launch_deposit_all(c->d, s);
  }
  // Reached sites per grain of the loaded claims.
  ge::launch_count_reached(c->d, s);
  HIPCHK(c, hipGetLastError());
  st = read_counters(c);
  if (st != GE_OK) return st;
  c->grain_host.clear();
  c->grain_c64.clear();
  c->grain_q64.clear();
  remember_grains(c, 0, S.n_grains, S.centre, S.quat);
  return error_status(c, c->host_cnt->err);
}

ge_status ge_load_state(ge_ctx* c, const ge_state_in* st_in) {
  if (!c || !st_in) return GE_EINVAL;
  return load_state(c, *st_in, nullptr, 0);
}

// ------------------------------------------------------ saved states ---
static_assert(sizeof(ge_state_header) == 128, "state header layout");
static_assert(sizeof(ge_state_grain) == 56 && sizeof(ge_state_site) == 72, "state record layout");
static_assert(sizeof(ge_state_particle) == 24 && sizeof(ge_state_claims) == 144,
              "state record layout");

namespace {

// 64-bit FNV-1a over little-endian 64-bit words.
uint64_t blob_checksum(const char* p, size_t bytes) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t k = 0; k + 8 <= bytes; k += 8) {
    uint64_t w;
    std::memcpy(&w, p + k, 8);
    h = (h ^ w) * 0x100000001b3ull;
  }
  return h;
}

size_t pad8(size_t v) { return (v + 7) / 8 * 8; }

// Section offsets of a blob with the header's counts; 0 when a count is
// negative or the sizes overflow.
struct BlobLayout {
  size_t grains, sites, particles, claims, total;
};
BlobLayout blob_layout(const ge_state_header& h) {
  BlobLayout L{};
  const int64_t n[4] = {h.n_grains, h.n_sites, h.n_particles, h.n_claim_bricks};
  const size_t rec[4] = {sizeof(ge_state_grain), sizeof(ge_state_site), sizeof(ge_state_particle),
                         sizeof(ge_state_claims)};
  size_t off = sizeof(ge_state_header), at[4];
  for (int k = 0; k < 4; ++k) {
    if (n[k] < 0 || (uint64_t)n[k] > (1ull << 40)) return BlobLayout{};
    at[k] = off;
    off = pad8(off + (size_t)n[k] * rec[k]);
  }
  L.grains = at[0];
  L.sites = at[1];
  L.particles = at[2];
  L.claims = at[3];
  L.total = off;
  return L;
}

}  // namespace

ge_status ge_state_check(const void* blob, size_t bytes, ge_state_header* hdr) {
  if (!blob || bytes < sizeof(ge_state_header)) return GE_EINVAL;
  ge_state_header h;
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != GE_STATE_MAGIC || h.version != GE_STATE_VERSION) return GE_EINVAL;
  if (h.bytes != bytes) return GE_EINVAL;
  const BlobLayout L = blob_layout(h);
  if (L.total == 0 || L.total != bytes) return GE_EINVAL;
  if (h.n_grains > INT32_MAX || h.n_sites > INT32_MAX || h.n_particles > UINT32_MAX ||
      h.n_claim_bricks > UINT32_MAX)
    return GE_EINVAL;
  if (blob_checksum((const char*)blob + sizeof(h), bytes - sizeof(h)) != h.checksum)
    return GE_EINVAL;
  if (hdr) *hdr = h;
  return GE_OK;
}

ge_status ge_save_state(ge_ctx* c, void* out, size_t out_bytes, size_t* needed) {
  if (!c) return GE_EINVAL;
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  if (c->host_cnt->err) return error_status(c, c->host_cnt->err);
  hipStream_t s = c->stream;
  const ge::Counters H = *c->host_cnt;
  // Particles and claim bricks are counted first (the size of the blob).
  uint32_t* counter = nullptr;
  HIPCHK(c, hipMalloc((void**)&counter, 8));
  HIPCHK(c, hipMemsetAsync(counter, 0, 8, s));
  ge::launch_export_particles(c->d, counter, nullptr, 0, nullptr, s);
  ge::launch_export_slots(c->d, counter + 1, nullptr, 0, s);
  uint32_t cnt[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(cnt, counter, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  ge_state_header h{};
  h.magic = GE_STATE_MAGIC;
  h.version = GE_STATE_VERSION;
  h.lambda0 = c->p.lambda0;
  for (int a = 0; a < 3; ++a) {
    h.lo[a] = c->p.lo[a];
    h.hi[a] = c->p.hi[a];
  }
  h.t = H.t;
  h.step = (int64_t)H.step;
  h.n_grains = H.n_grains;
  h.n_sites = c->n_sites;
  h.n_particles = cnt[0];
  h.n_claim_bricks = cnt[1];
  const BlobLayout L = blob_layout(h);
  h.bytes = L.total;
  if (needed) *needed = L.total;
  if (!out || out_bytes < L.total) {
    (void)hipFree(counter);
    return GE_OK;
  }
  char* o = (char*)out;
  std::memset(o, 0, L.total);
  // Grains: FP64 definitions from the host, or from the site a grain was
  // nucleated at.
  std::vector<int32_t> gsite(H.n_grains);
  if (H.n_grains)
    HIPCHK(c, hipMemcpyAsync(gsite.data(), c->d.gsite, 4 * (size_t)H.n_grains,
                             hipMemcpyDeviceToHost, s));
  std::vector<uint32_t> sst(c->n_sites);
  if (c->n_sites)
    HIPCHK(c, hipMemcpyAsync(sst.data(), c->d.sstate, 4 * (size_t)c->n_sites,
                             hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (uint32_t g = 0; g < H.n_grains; ++g) {
    ge_state_grain r{};
    if (g < c->grain_host.size() && c->grain_host[g]) {
      std::memcpy(r.centre, &c->grain_c64[3 * (size_t)g], sizeof(r.centre));
      std::memcpy(r.quat, &c->grain_q64[4 * (size_t)g], sizeof(r.quat));
    } else if (gsite[g] >= 0 && (uint32_t)gsite[g] < c->n_sites) {
      const size_t i = (size_t)gsite[g];
      std::memcpy(r.centre, &c->site_xyz[3 * i], sizeof(r.centre));
      std::memcpy(r.quat, &c->site_q64[4 * i], sizeof(r.quat));
    } else {
      (void)hipFree(counter);
      return fail(c, GE_ESTATE, "grain without a known definition");
    }
    std::memcpy(o + L.grains + g * sizeof(r), &r, sizeof(r));
  }
  for (uint32_t i = 0; i < c->n_sites; ++i) {
    ge_state_site r{};
    std::memcpy(r.xyz, &c->site_xyz[3 * (size_t)i], sizeof(r.xyz));
    r.dT_nuc = c->site_dT64[i];
    std::memcpy(r.quat, &c->site_q64[4 * (size_t)i], sizeof(r.quat));
    r.state = (int32_t)sst[i];
    std::memcpy(o + L.sites + i * sizeof(r), &r, sizeof(r));
  }
  // Particles (export records, then the saved form) and claim bricks
  // (written by the device in their saved form), staged on the device.
  const size_t pbytes = (size_t)cnt[0] * sizeof(ge_particle_rec);
  const size_t cbytes = (size_t)cnt[1] * sizeof(ge_state_claims);
  char* stage = nullptr;
  HIPCHK(c, hipMalloc((void**)&stage, std::max<size_t>(std::max(pbytes, cbytes), 64)));
  std::vector<ge_particle_rec> prec(cnt[0]);
  if (cnt[0]) {
    HIPCHK(c, hipMemsetAsync(counter, 0, 4, s));
    ge::launch_export_particles(c->d, counter, stage, cnt[0], nullptr, s);
    HIPCHK(c, hipMemcpyAsync(prec.data(), stage, pbytes, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (cnt[1]) {
    HIPCHK(c, hipMemsetAsync(counter, 0, 4, s));
    ge::launch_export_slots(c->d, counter, stage, cnt[1], s);
    HIPCHK(c, hipMemcpyAsync(o + L.claims, stage, cbytes, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  (void)hipFree(stage);
  (void)hipFree(counter);
  for (uint32_t k = 0; k < cnt[0]; ++k) {
    const ge_particle_rec& q = prec[k];
    ge_state_particle r{};
    r.s = q.s;
    r.grain = q.grain;
    std::memcpy(r.site, q.site, sizeof(r.site));
    r.dir = q.dir;
    r.state = q.state;
    std::memcpy(o + L.particles + (size_t)k * sizeof(r), &r, sizeof(r));
  }
  h.checksum = blob_checksum(o + sizeof(h), L.total - sizeof(h));
  std::memcpy(o, &h, sizeof(h));
  return GE_OK;
}

ge_status ge_restore_state(ge_ctx* c, const void* blob, size_t bytes) {
  if (!c) return GE_EINVAL;
  ge_state_header h;
  if (ge_state_check(blob, bytes, &h) != GE_OK) return fail(c, GE_EINVAL, "not a valid saved state");
  if (h.lambda0 != c->p.lambda0) return fail(c, GE_EINVAL, "saved with another lambda0");
  for (int a = 0; a < 3; ++a)
    if (h.lo[a] != c->p.lo[a] || h.hi[a] != c->p.hi[a]) return fail(c, GE_EINVAL, "saved with another box");
  const BlobLayout L = blob_layout(h);
  const char* b = (const char*)blob;
  // Nucleation sites: registered from the blob, or equal to it.
  std::vector<double> xyz(3 * (size_t)h.n_sites), dTn((size_t)h.n_sites), q(4 * (size_t)h.n_sites);
  std::vector<int32_t> sst((size_t)h.n_sites);
  for (int64_t i = 0; i < h.n_sites; ++i) {
    ge_state_site r;
    std::memcpy(&r, b + L.sites + (size_t)i * sizeof(r), sizeof(r));
    std::memcpy(&xyz[3 * i], r.xyz, sizeof(r.xyz));
    dTn[i] = r.dT_nuc;
    std::memcpy(&q[4 * i], r.quat, sizeof(r.quat));
    sst[i] = r.state;
    if (r.state < GE_SITE_DORMANT || r.state > GE_SITE_ENGULFED) return fail(c, GE_EINVAL, "bad site state");
  }
  if (c->n_sites == 0 && h.n_sites > 0) {
    const ge_status st = ge_nucleate(c, (int32_t)h.n_sites, xyz.data(), dTn.data(), q.data());
    if (st != GE_OK) return st;
  } else if ((int64_t)c->n_sites != h.n_sites || c->site_xyz != xyz || c->site_dT64 != dTn ||
             c->site_q64 != q) {
    return fail(c, GE_EINVAL, "registered sites differ from the saved ones");
  }
  std::vector<double> gc(3 * (size_t)h.n_grains), gq(4 * (size_t)h.n_grains);
  for (int64_t g = 0; g < h.n_grains; ++g) {
    ge_state_grain r;
    std::memcpy(&r, b + L.grains + (size_t)g * sizeof(r), sizeof(r));
    std::memcpy(&gc[3 * g], r.centre, sizeof(r.centre));
    std::memcpy(&gq[4 * g], r.quat, sizeof(r.quat));
  }
  const size_t np = (size_t)h.n_particles;
  std::vector<int32_t> pg(np), ps(3 * np), pd(np), pst(np);
  std::vector<float> pss(np);
  for (size_t k = 0; k < np; ++k) {
    ge_state_particle r;
    std::memcpy(&r, b + L.particles + k * sizeof(r), sizeof(r));
    pg[k] = (int32_t)r.grain;
    std::memcpy(&ps[3 * k], r.site, sizeof(r.site));
    pd[k] = r.dir;
    pss[k] = r.s;
    pst[k] = r.state;
  }
  for (int64_t k = 0; k < h.n_claim_bricks; ++k) {
    ge_state_claims r;
    std::memcpy(&r, b + L.claims + (size_t)k * sizeof(r), sizeof(r));
    if (r.grain >= (uint64_t)h.n_grains) return fail(c, GE_EINVAL, "bad claim grain");
    for (int a = 0; a < 3; ++a)
      if (std::abs((int64_t)r.brick[a]) * 8 > MAX_SITE_RANGE + 8) return fail(c, GE_EINVAL, "claim site out of range");
  }
  ge_state_in S{};
  S.n_grains = (int32_t)h.n_grains;
  S.centre = gc.data();
  S.quat = gq.data();
  S.n_particles = (int64_t)np;
  S.grain = pg.data();
  S.site = ps.data();
  S.dir = pd.data();
  S.s = pss.data();
  S.state = pst.data();
  S.n_claims = 0;
  S.n_sites = (int32_t)h.n_sites;
  S.site_state = sst.data();
  S.t = h.t;
  S.step = h.step;
  return load_state(c, S, b + L.claims, h.n_claim_bricks);
}

ge_status ge_set_melting(ge_ctx* c, int32_t on) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (on && c->adj.valid && c->d.tagA) return fail(c, GE_ESTATE, "an adjoint run is being recorded");
  c->d.melting = on ? 1 : 0;
  // Reached sites per grain (kept step by step while melting is on).
  if (on) {
    ge::launch_count_reached(c->d, c->stream);
    HIPCHK(c, hipGetLastError());
  }
  return sync_dev(c);
}

ge_status ge_set_deposition_grid(ge_ctx* c, const int32_t n[3], const double origin[3],
                                 const double spacing[3]) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  Dev& d = c->d;
  if (!n || n[0] == 0 || n[1] == 0 || n[2] == 0) {
    d.gcnt = nullptr;
    c->dep_nodes = 0;
    return sync_dev(c);
  }
  if (!origin || !spacing) return fail(c, GE_EINVAL, "missing grid geometry");
  uint64_t nodes = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > c->p.field_n[a]) return fail(c, GE_EINVAL, "deposition grid larger than field_n");
    if (!std::isfinite(origin[a]) || !(spacing[a] > 0) || !std::isfinite(spacing[a]))
      return fail(c, GE_EINVAL, "bad deposition grid geometry");
    nodes *= (uint64_t)n[a];
  }
  d.gcnt = (uint32_t*)(c->ws + c->lay.gcnt);
  for (int a = 0; a < 3; ++a) {
    d.gn[a] = n[a];
    d.go[a] = (float)origin[a];
    d.ginv[a] = (float)(1.0 / spacing[a]);
  }
  c->dep_nodes = nodes;
  c->dep_cell_volume = spacing[0] * spacing[1] * spacing[2];
  HIPCHK(c, hipMemsetAsync(d.gcnt, 0, 4 * nodes, c->stream));
  ge::launch_deposit_all(d, c->stream);
  HIPCHK(c, hipGetLastError());
  return sync_dev(c);
}

// ------------------------------------------------------------- model ----
ge_status ge_set_model(ge_ctx* c, const double a[2], const double b[2], double theta,
                       int32_t branching) {
  if (!c || !a || !b) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  ge_params p = c->p;
  p.a[0] = a[0];
  p.a[1] = a[1];
  p.b[0] = b[0];
  p.b[1] = b[1];
  p.theta = theta;
  p.branching = branching ? 1 : 0;
  if (const char* why = check_params(&p)) return fail(c, GE_EINVAL, why);
  c->p = p;
  Dev& d = c->d;
  d.ka[0] = (float)p.a[0];
  d.ka[1] = (float)p.a[1];
  d.kb[0] = (float)p.b[0];
  d.kb[1] = (float)p.b[1];
  d.kin_poly = (p.b[0] == 2.0 && p.b[1] == 3.0) ? 1 : 0;
  d.theta = (float)p.theta;
  d.branching = p.branching;
  return sync_dev(c);
}

// ----------------------------------------------------------- adjoint ----
// Layout of the caller's adjoint workspace for n_cap tracked particles.
static size_t adj_layout(ge_ctx::Adj& A, uint64_t n_cap, int32_t n_steps, int32_t K) {
  size_t off = 0;
  auto put = [&](uint64_t bytes) {
    const size_t o = off;
    off += align_up(std::max<size_t>((size_t)bytes, 1));
    return o;
  };
  const uint64_t nck = ((uint64_t)n_steps + (uint64_t)K - 1) / (uint64_t)K;
  A.tagA = put(4 * n_cap);
  A.tagB = put(4 * n_cap);
  A.rec = put(16 * n_cap);
  A.nact = put(4 * n_cap);
  A.sfin = put(4 * n_cap);
  A.ck = put(4 * n_cap * nck);
  A.seg = put(4 * n_cap * (uint64_t)K);
  A.xN = put(12 * n_cap);
  A.dldx = put(12 * n_cap);
  A.linc = put(4 * (uint64_t)n_steps);
  A.part = put(24 * (uint64_t)ge::ADJ_BLOCKS);
  A.grad = put(24);
  A.mis = put(4);
  A.total = off;
  return off;
}

ge_status ge_adjoint_workspace_size(const ge_ctx* c, int32_t n_steps, int32_t ckpt_every,
                                    size_t* bytes) {
  if (!c || !bytes || n_steps < 1 || ckpt_every < 1) return GE_EINVAL;
  ge_ctx::Adj A;
  *bytes = adj_layout(A, (uint64_t)c->p.cap_particles, n_steps, ckpt_every);
  return GE_OK;
}

ge_status ge_adjoint_forward(ge_ctx* c, double dt, int32_t n_steps, int32_t ckpt_every,
                             void* workspace, size_t bytes, int64_t* n_tracked) {
  if (!c) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (!(std::isfinite(dt) && dt > 0) || n_steps < 1 || ckpt_every < 1 || !workspace)
    return fail(c, GE_EINVAL, "bad adjoint arguments");
  if (((uintptr_t)workspace) % ALIGN) return fail(c, GE_EINVAL, "adjoint workspace not 256-byte aligned");
  if (c->d.branching) return fail(c, GE_EINVAL, "the recorded run needs branching off");
  if (c->d.melting) return fail(c, GE_EINVAL, "the recorded run needs melting off");
  if (c->field.kind == GE_FIELD_ROSENTHAL)
    return fail(c, GE_EINVAL, "the recorded run needs a field that is fixed in time (not ROSENTHAL)");
  ge_ctx::Adj A;
  if (adj_layout(A, (uint64_t)c->p.cap_particles, n_steps, ckpt_every) > bytes)
    return fail(c, GE_EINVAL, "adjoint workspace too small");
  ge_status st = read_counters(c);
  if (st != GE_OK) return st;
  if ((st = error_status(c, c->host_cnt->err)) != GE_OK) return st;
  const uint32_t n = c->host_cnt->n_active;  // records of the active store
  char* w = (char*)workspace;
  A.ws = w;
  A.n = n;
  A.n_steps = n_steps;
  A.K = ckpt_every;
  A.dt = (float)dt;
  c->adj = A;
  c->adj.valid = false;
  Dev& d = c->d;
  d.tagA = (uint32_t*)(w + A.tagA);
  d.tagB = (uint32_t*)(w + A.tagB);
  d.adj_rec = (uint4*)(w + A.rec);
  d.adj_nact = (int32_t*)(w + A.nact);
  d.adj_sfin = (float*)(w + A.sfin);
  d.adj_ck = (float*)(w + A.ck);
  d.adj_ncap = n;
  d.adj_K = ckpt_every;
  d.adj_step0 = c->host_cnt->step;
  d.adj_linc = (float*)(w + A.linc);
  if ((st = sync_dev(c)) != GE_OK) return st;
  hipStream_t s = c->stream;
  ge::launch_adj_init(d, n, n_steps, s);
  ge::launch_reset_stats(d, s);
  for (int32_t k = 0; k < n_steps; ++k) step_once(c, dt);
  ge::launch_adj_final(d, s);
  ge::launch_adj_positions(d, n, (float*)(w + A.xN), s);
  d.tagA = d.tagB = nullptr;  // later steps run untracked
  HIPCHK(c, hipGetLastError());
  if ((st = sync_dev(c)) != GE_OK) return st;
  st = read_counters(c);
  if (st != GE_OK) return st;
  if ((st = error_status(c, c->host_cnt->err)) != GE_OK) return st;
  c->adj.valid = true;
  if (n_tracked) *n_tracked = (int64_t)n;
  return GE_OK;
}

ge_status ge_adjoint_positions(ge_ctx* c, float* xN, size_t bytes, int32_t on_device) {
  if (!c || !xN) return GE_EINVAL;
  if (!c->adj.valid) return fail(c, GE_ESTATE, "no recorded run");
  const size_t need = 12 * (size_t)c->adj.n;
  if (bytes < need) return fail(c, GE_EINVAL, "output too small");
  HIPCHK(c, hipMemcpyAsync(xN, c->adj.ws + c->adj.xN, need,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

ge_status ge_adjoint_tracked(ge_ctx* c, ge_adjoint_rec* out, size_t bytes) {
  if (!c || !out) return GE_EINVAL;
  if (!c->adj.valid) return fail(c, GE_ESTATE, "no recorded run");
  const size_t n = c->adj.n;
  if (bytes < n * sizeof(ge_adjoint_rec)) return fail(c, GE_EINVAL, "output too small");
  std::vector<uint32_t> rec(4 * n);
  std::vector<int32_t> nact(n);
  std::vector<float> sfin(n);
  const char* w = c->adj.ws;
  hipStream_t s = c->stream;
  if (n) {
    HIPCHK(c, hipMemcpyAsync(rec.data(), w + c->adj.rec, 16 * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(nact.data(), w + c->adj.nact, 4 * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(sfin.data(), w + c->adj.sfin, 4 * n, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i) {
    const uint32_t* r = &rec[4 * i];
    ge_adjoint_rec& o = out[i];
    std::memset(&o, 0, sizeof(o));
    std::memcpy(&o.s0, &r[0], 4);
    o.grain = r[1] >> 3;
    o.dir = (uint8_t)(r[1] & 7u);
    o.site[0] = (int16_t)(r[2] & 0xFFFFu);
    o.site[1] = (int16_t)(r[2] >> 16);
    o.site[2] = (int16_t)(r[3] & 0xFFFFu);
    o.state0 = (uint8_t)((r[3] >> 16) & 3u);
    o.nact = nact[i];
    o.s_final = sfin[i];
  }
  return GE_OK;
}

ge_status ge_adjoint_backward(ge_ctx* c, const float* dLdx, int32_t on_device, double grad[3]) {
  if (!c || !dLdx || !grad) return GE_EINVAL;
  if (c->dead) return fail(c, GE_ESTATE, "context unusable after an earlier error");
  if (!c->adj.valid) return fail(c, GE_ESTATE, "no recorded run");
  const ge_ctx::Adj& A = c->adj;
  char* w = A.ws;
  hipStream_t s = c->stream;
  const float* g = dLdx;
  if (!on_device) {
    if (A.n) HIPCHK(c, hipMemcpyAsync(w + A.dldx, dLdx, 12 * (size_t)A.n, hipMemcpyHostToDevice, s));
    g = (const float*)(w + A.dldx);
  }
  HIPCHK(c, hipMemsetAsync(w + A.mis, 0, 4, s));
  ge::launch_adj_backward(c->d, A.n, A.n_steps, A.K, (const float*)(w + A.linc), A.dt, g,
                          (float*)(w + A.seg), (double*)(w + A.part), (double*)(w + A.grad),
                          (uint32_t*)(w + A.mis), s);
  double out[3];
  uint32_t mis = 0;
  HIPCHK(c, hipMemcpyAsync(out, w + A.grad, 24, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&mis, w + A.mis, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  HIPCHK(c, hipGetLastError());
  if (mis) return fail(c, GE_ESTATE, "the replay differs from the recorded run (model, field or grains changed)");
  for (int k = 0; k < 3; ++k) grad[k] = out[k];
  return GE_OK;
}

}  // extern "C"

// ------------------------------------------------------------- batches ---
// Many contexts advanced by one launch per phase: each launch gives every
// context a share of its blocks.  The contexts live in one workspace so that
// their tables can hold offsets from its base.
struct ge_batch {
  std::vector<ge_ctx*> mem;
  std::vector<size_t> mem_off;
  char* base = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  uint32_t cap[ge::BS_N] = {0};      // map entries per site
  uint32_t T[ge::BS_N] = {0};        // blocks of the shared sites (0: fixed sites)
  size_t off_tab = 0, off_map[ge::BS_N] = {0}, off_gsz[ge::BS_N] = {0};
  ge::BatchLaunch L{};
  std::vector<Dev> htab;
  std::vector<uint32_t> hmap, hgsz;
  bool use_graphs = true;
  hipGraphExec_t gexec = nullptr;
  bool gvalid = false;
  double gdt = 0.0;
  uint32_t gtotal[ge::BS_N] = {0};
  hipStream_t cap_stream = nullptr;
  int32_t R = 16;
  std::string err;
};

namespace {

constexpr uint32_t BATCH_MAX_BLOCKS = 65536;  // blocks of one shared launch

// Tunable kernel of each shared site (-1: fixed site).
const int SITE_TK[ge::BS_N] = {-1, ge::TK_ADVANCE, -1, ge::TK_BRANCH, -1,
                               ge::TK_CELLSCAN, ge::TK_SCATTER, ge::TK_CHILDREN, ge::TK_DIRTY,
                               ge::TK_CONTAIN, ge::TK_STOPLINK, -1, -1, -1};

uint32_t tiles_of(const Dev& d) {
  return (uint32_t)((d.n_bricks + ge::SCAN_TILE_HOST - 1) / ge::SCAN_TILE_HOST);
}
uint32_t grid_cap(uint64_t n, uint32_t cap) {
  uint64_t g = (n + 255) / 256;
  g = std::max<uint64_t>(g, 1);
  return (uint32_t)std::min<uint64_t>(g, cap);
}

struct BatchLayout {
  std::vector<size_t> mem_off, mem_size;
  size_t off_tab, off_map[ge::BS_N], off_gsz[ge::BS_N], total;
  uint32_t cap[ge::BS_N];
};

const char* batch_layout(int32_t n, const ge_params* params, BatchLayout& B) {
  if (n < 1 || (uint32_t)n > ge::BATCH_MAX || !params) return "bad batch size";
  size_t off = 0;
  uint64_t tiles = 0, resample = 0, nuc = 0;
  for (int32_t i = 0; i < n; ++i) {
    size_t sz = 0;
    if (ge_workspace_size(&params[i], &sz) != GE_OK) return "invalid member parameters";
    B.mem_off.push_back(off);
    B.mem_size.push_back(sz);
    off += align_up(sz);
    const Geometry g = geometry(&params[i]);
    tiles += (g.n_bricks + ge::SCAN_TILE_HOST - 1) / ge::SCAN_TILE_HOST;
    const uint64_t nodes = (uint64_t)params[i].field_n[0] * params[i].field_n[1] * params[i].field_n[2];
    if (nodes) resample += grid_cap(nodes, 8192);
    if (params[i].cap_sites > 0) nuc += grid_cap((uint64_t)params[i].cap_sites, 1024);
  }
  // A shared launch has max(T, 8 n) blocks, T <= BATCH_MAX_BLOCKS.
  const uint32_t share = std::max<uint32_t>(BATCH_MAX_BLOCKS, 8u * (uint32_t)n);
  for (int k = 0; k < ge::BS_N; ++k) B.cap[k] = share;
  B.cap[ge::BS_ONE] = (uint32_t)n;
  B.cap[ge::BS_NUCFIRE] = (uint32_t)n;
  B.cap[ge::BS_TILES] = (uint32_t)tiles;
  B.cap[ge::BS_RESAMPLE] = (uint32_t)std::max<uint64_t>(resample, 1);
  B.cap[ge::BS_NUCTEST] = (uint32_t)std::max<uint64_t>(nuc, 1);
  B.off_tab = off;
  off += align_up(sizeof(Dev) * (size_t)n);
  for (int k = 0; k < ge::BS_N; ++k) {  // the maps, contiguous
    B.off_map[k] = off;
    off += align_up(4 * (size_t)B.cap[k]);
  }
  for (int k = 0; k < ge::BS_N; ++k) B.off_gsz[k] = off + 4 * (size_t)k * (size_t)n;
  off += align_up(4 * (size_t)ge::BS_N * (size_t)n);  // then the per-context block counts
  B.total = off;
  return nullptr;
}

ge_status bfail(ge_batch* b, ge_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

// Per-context blocks of every site for the current particle counts, the
// tables (pointers as offsets, writer grids of the shared per-block lists set
// to the contexts' shares) and their upload.
ge_status batch_bind(ge_batch* b) {
  const uint32_t n = (uint32_t)b->mem.size();
  std::vector<double> w(n);
  double wsum = 0;
  for (uint32_t m = 0; m < n; ++m) {
    ge_ctx* c = b->mem[m];
    if (c->dead) return bfail(b, GE_ESTATE, "a member context is unusable after an earlier error");
    ge_status st = read_counters(c);
    if (st != GE_OK) return bfail(b, st, c->err);
    w[m] = (double)c->host_cnt->n_active + 64.0;
    wsum += w[m];
  }
  std::vector<uint32_t> g(n);
  for (int k = 0; k < ge::BS_N; ++k) {
    for (uint32_t m = 0; m < n; ++m) {
      const Dev& d = b->mem[m]->d;
      uint32_t v = 0;
      switch (k) {
        case ge::BS_ONE: v = 1; break;
        case ge::BS_TILES: v = tiles_of(d); break;
        case ge::BS_RESAMPLE:
          v = b->mem[m]->field.kind == GE_FIELD_ROSENTHAL
                  ? grid_cap((uint64_t)d.fn[0] * d.fn[1] * d.fn[2], 8192) : 0;
          break;
        case ge::BS_NUCTEST: v = d.n_sites ? grid_cap(d.n_sites, 1024) : 0; break;
        case ge::BS_NUCFIRE: v = d.n_sites ? 1 : 0; break;
        default: break;
      }
      g[m] = v;
    }
    if (SITE_TK[k] >= 0 || k == ge::BS_RESORT) {
      // Shared site: 8 blocks per context, the rest in units of 8 by weight
      // (largest remainders), T blocks in all (at least 8 per context).
      const uint32_t units = std::max<uint32_t>(b->T[k] / 8u, n);
      const uint32_t extra = units - n;
      std::vector<std::pair<double, uint32_t>> frac(n);
      uint32_t given = 0;
      for (uint32_t m = 0; m < n; ++m) {
        const double q = extra * w[m] / wsum;
        const uint32_t u = (uint32_t)q;
        g[m] = 8u * (1u + u);
        given += u;
        frac[m] = {q - u, m};
      }
      std::sort(frac.begin(), frac.end(), [](auto& x, auto& y) {
        return x.first != y.first ? x.first > y.first : x.second < y.second;
      });
      for (uint32_t r = 0; given < extra; ++r, ++given) g[frac[r % n].second] += 8u;
      // Per-block lists hold at most STREAM_GRID regions per context.
      for (uint32_t m = 0; m < n; ++m) g[m] = std::min<uint32_t>(g[m], ge::STREAM_GRID);
    }
    uint32_t total = 0;
    for (uint32_t m = 0; m < n; ++m) {
      if ((uint64_t)total + g[m] > b->cap[k]) return bfail(b, GE_EINVAL, "batch site capacity");
      for (uint32_t v = 0; v < g[m]; ++v) b->hmap[(b->off_map[k] - b->off_map[0]) / 4 + total + v] = m | (v << 12);
      b->hgsz[(size_t)k * n + m] = g[m];
      total += g[m];
    }
    b->L.site[k].total = total;
    if (SITE_TK[k] == ge::TK_ADVANCE || SITE_TK[k] == ge::TK_CONTAIN)
      for (uint32_t m = 0; m < n; ++m) b->htab[m].sched[SITE_TK[k]] = g[m];
  }
  for (uint32_t m = 0; m < n; ++m) {
    const Dev& d = b->mem[m]->d;
    Dev& t = b->htab[m];
    const uint32_t sa = t.sched[ge::TK_ADVANCE], sc = t.sched[ge::TK_CONTAIN];
    t = d;
    t.sched[ge::TK_ADVANCE] = sa;
    t.sched[ge::TK_CONTAIN] = sc;
    if (t.tagA || t.tagB) return bfail(b, GE_ESTATE, "a member is recording an adjoint run");
    if (t.melting) return bfail(b, GE_EINVAL, "melting is not available in batched steps");
#define GE_TO_OFFSET(f) \
    t.f = t.f ? (decltype(t.f))((uintptr_t)((char*)t.f - b->base)) : (decltype(t.f))ge::NULL_OFFSET;
    GE_DEV_POINTERS(GE_TO_OFFSET)
#undef GE_TO_OFFSET
  }
  hipStream_t s = b->stream;
  char* w0 = b->base;
  if (hipMemcpyAsync(w0 + b->off_tab, b->htab.data(), sizeof(Dev) * n, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(w0 + b->off_map[0], b->hmap.data(), 4 * b->hmap.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemcpyAsync(w0 + b->off_gsz[0], b->hgsz.data(), 4 * b->hgsz.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bfail(b, GE_EDEVICE, "batch table upload failed");
  return GE_OK;
}

ge_status batch_graph(ge_batch* b, double dt) {
  bool same = b->gvalid && b->gdt == dt;
  for (int k = 0; k < ge::BS_N && same; ++k) same = b->gtotal[k] == b->L.site[k].total;
  if (same) return GE_OK;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->gvalid = false;
  if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return bfail(b, GE_EDEVICE, "capture stream");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int32_t k = 0; k < b->R; ++k) ge::launch_batch_step(b->L, dt, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return bfail(b, GE_EDEVICE, std::string("batch graph: ") + hipGetErrorString(e));
  b->gvalid = true;
  b->gdt = dt;
  for (int k = 0; k < ge::BS_N; ++k) b->gtotal[k] = b->L.site[k].total;
  return GE_OK;
}

}  // namespace

extern "C" {

ge_status ge_batch_workspace_size(int32_t n, const ge_params* params, size_t* bytes) {
  if (!bytes) return GE_EINVAL;
  BatchLayout B;
  if (batch_layout(n, params, B)) return GE_EINVAL;
  *bytes = B.total;
  return GE_OK;
}

ge_status ge_batch_create(int32_t n, const ge_params* params, void* workspace, size_t bytes,
                          void* stream, ge_batch** out) {
  if (!out || !workspace) return GE_EINVAL;
  *out = nullptr;
  BatchLayout B;
  if (batch_layout(n, params, B)) return GE_EINVAL;
  if (bytes < B.total || ((uintptr_t)workspace) % ALIGN) return GE_EINVAL;
  ge_batch* b = new ge_batch();
  b->base = (char*)workspace;
  b->bytes = bytes;
  b->stream = (hipStream_t)stream;
  for (int32_t i = 0; i < n; ++i) {
    ge_ctx* c = nullptr;
    const ge_status st = ge_create(&params[i], b->base + B.mem_off[i], B.mem_size[i], stream, &c);
    if (st != GE_OK) {
      ge_batch_destroy(b);
      return st;
    }
    b->mem.push_back(c);
    b->mem_off.push_back(B.mem_off[i]);
  }
  b->off_tab = B.off_tab;
  for (int k = 0; k < ge::BS_N; ++k) {
    b->off_map[k] = B.off_map[k];
    b->off_gsz[k] = B.off_gsz[k];
    b->cap[k] = B.cap[k];
    const int tk = SITE_TK[k];
    b->T[k] = tk >= 0 ? b->mem[0]->d.sched[tk] : (k == ge::BS_RESORT ? ge::STREAM_GRID : 0);
  }
  // One host staging array for all maps, in the workspace's order.
  b->hmap.assign((b->off_map[ge::BS_N - 1] - b->off_map[0]) / 4 + b->cap[ge::BS_N - 1], 0u);
  b->hgsz.assign((size_t)ge::BS_N * n, 0u);
  b->htab.resize(n);
  b->L.tab = (const Dev*)(b->base + b->off_tab);
  b->L.base = b->base;
  for (int k = 0; k < ge::BS_N; ++k) {
    b->L.site[k].map = (const uint32_t*)(b->base + b->off_map[k]);
    b->L.site[k].gsz = (const uint32_t*)(b->base + b->off_gsz[0]) + (size_t)k * n;
  }
  b->R = b->mem[0]->resort_every;
  b->L.any_periodic = 0;
  for (ge_ctx* m : b->mem) b->L.any_periodic |= m->d.periodic != 0 ? 1 : 0;
  *out = b;
  return GE_OK;
}

ge_status ge_batch_destroy(ge_batch* b) {
  if (!b) return GE_EINVAL;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (ge_ctx* c : b->mem) ge_destroy(c);
  delete b;
  return GE_OK;
}

ge_status ge_batch_member(ge_batch* b, int32_t i, ge_ctx** out) {
  if (!b || !out || i < 0 || (size_t)i >= b->mem.size()) return GE_EINVAL;
  *out = b->mem[(size_t)i];
  return GE_OK;
}

const char* ge_batch_last_error(const ge_batch* b) { return b ? b->err.c_str() : ""; }

ge_status ge_batch_use_graphs(ge_batch* b, int32_t on) {
  if (!b) return GE_EINVAL;
  b->use_graphs = on != 0;
  return GE_OK;
}

ge_status ge_batch_step(ge_batch* b, double dt, int32_t n_steps, ge_step_stats* stats) {
  if (!b) return GE_EINVAL;
  if (!(std::isfinite(dt) && dt > 0) || n_steps < 0) return bfail(b, GE_EINVAL, "bad dt or n_steps");
  ge_status st = batch_bind(b);
  if (st != GE_OK) return st;
  hipStream_t s = b->stream;
  ge::launch_batch_reset_stats(b->L, s);
  int32_t k = 0;
  if (b->use_graphs && n_steps >= 2 * b->R) {
    if ((st = batch_graph(b, dt)) != GE_OK) return st;
    const int32_t reps = n_steps / b->R;
    for (int32_t r = 0; r < reps; ++r)
      if (hipGraphLaunch(b->gexec, s) != hipSuccess) return bfail(b, GE_EDEVICE, "graph launch");
    k = reps * b->R;
  }
  for (; k < n_steps; ++k) ge::launch_batch_step(b->L, dt, s);
  if (hipGetLastError() != hipSuccess) return bfail(b, GE_EDEVICE, "batch launch");
  ge_status worst = GE_OK;
  for (size_t m = 0; m < b->mem.size(); ++m) {
    ge_ctx* c = b->mem[m];
    st = read_counters(c);
    if (st != GE_OK) return bfail(b, st, c->err);
    c->hstep = c->host_cnt->step;
    if (stats) fill_stats(c, &stats[m]);
    st = error_status(c, c->host_cnt->err);
    if (st != GE_OK && worst == GE_OK) {
      worst = st;
      b->err = "member " + std::to_string(m) + ": " + c->err;
    }
  }
  return worst;
}

ge_status ge_batch_get_blocks(ge_batch* b, int32_t* blocks) {
  if (!b || !blocks) return GE_EINVAL;
  for (int t = 0; t < GE_N_TUNABLE; ++t) blocks[t] = 0;
  for (int k = 0; k < ge::BS_N; ++k)
    if (SITE_TK[k] >= 0) blocks[SITE_TK[k]] = (int32_t)b->T[k];
  return GE_OK;
}

ge_status ge_batch_set_blocks(ge_batch* b, const int32_t* blocks) {
  if (!b || !blocks) return GE_EINVAL;
  for (int t = 0; t < GE_N_TUNABLE; ++t)
    if (blocks[t] < 0 || blocks[t] > (int32_t)BATCH_MAX_BLOCKS) return bfail(b, GE_EINVAL, "blocks out of range");
  for (int k = 0; k < ge::BS_N; ++k)
    if (SITE_TK[k] >= 0 && blocks[SITE_TK[k]] > 0) b->T[k] = (uint32_t)blocks[SITE_TK[k]];
  return GE_OK;
}

ge_status ge_batch_autotune(ge_batch* b, double dt, int32_t steps_per_trial, void* snapshot,
                            size_t snapshot_bytes, int32_t* blocks_out) {
  if (!b || steps_per_trial < 1) return GE_EINVAL;
  if (snapshot && snapshot_bytes < b->bytes)
    return bfail(b, GE_EINVAL, "snapshot smaller than the batch workspace");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return bfail(b, GE_EDEVICE, "device query");
  const uint32_t n = (uint32_t)b->mem.size();
  std::vector<uint32_t> cand;
  for (int per = 1; per <= 8; ++per) {
    uint32_t g = (uint32_t)std::max(per * std::max(cus, 1), (int)(8 * n));
    g = g / 8u * 8u;
    if (cand.empty() || cand.back() != g) cand.push_back(g);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return bfail(b, GE_EDEVICE, "events");
  ge_status st = GE_OK;
  std::vector<uint64_t> hstep0;
  for (ge_ctx* c : b->mem) hstep0.push_back(c->hstep);
  auto copy = [&](void* dst, const void* src) -> ge_status {
    return hipMemcpyAsync(dst, src, b->bytes, hipMemcpyDeviceToDevice, b->stream) == hipSuccess
               ? GE_OK
               : bfail(b, GE_EDEVICE, "autotune snapshot");
  };
  // The snapshot covers the launch tables of the batch too: a restore comes
  // before batch_bind, which writes the tables of the trial's totals.
  if (snapshot) st = copy(snapshot, b->base);
  for (int k = 0; k < ge::BS_N && st == GE_OK; ++k) {
    if (SITE_TK[k] < 0) continue;
    uint32_t best = b->T[k];
    double best_cost = INFINITY;
    for (uint32_t g : cand) {
      b->T[k] = g;
      if (snapshot && (st = copy(b->base, snapshot)) != GE_OK) break;
      if ((st = batch_bind(b)) != GE_OK) break;
      (void)hipEventRecord(e0, b->stream);
      for (int32_t r = 0; r < steps_per_trial; ++r) ge::launch_batch_step(b->L, dt, b->stream);
      (void)hipEventRecord(e1, b->stream);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = bfail(b, GE_EDEVICE, "autotune step");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      uint64_t adv = 0;
      for (ge_ctx* c : b->mem) {
        if ((st = read_counters(c)) != GE_OK) break;
        adv += c->host_cnt->n_active;
      }
      if (st != GE_OK) break;
      const double cost = ms / (double)std::max<uint64_t>(adv, 1);
      if (cost < best_cost) {
        best_cost = cost;
        best = g;
      }
    }
    b->T[k] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (snapshot && st == GE_OK) {
    st = copy(b->base, snapshot);
    for (size_t i = 0; i < b->mem.size(); ++i) b->mem[i]->hstep = hstep0[i];
    if (st == GE_OK) st = batch_bind(b);
  }
  for (ge_ctx* c : b->mem)
    if (read_counters(c) == GE_OK) c->hstep = c->host_cnt->step;
  if (st != GE_OK) return st;
  return blocks_out ? ge_batch_get_blocks(b, blocks_out) : GE_OK;
}

}  // extern "C"
