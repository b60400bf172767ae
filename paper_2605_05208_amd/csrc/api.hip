// api.hip -- C-ABI entry points of libmdvrp (host side).
//
// Validation runs on the host before any launch; device state is carved out of
// caller-provided workspaces; launches go to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mdvrp.h"
#include "kernels.h"

using namespace mdvrp;

namespace {

thread_local std::string g_err;

mdvrp_status fail(mdvrp_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mdvrp_status fail(mdvrp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MDVRP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over a caller workspace; with base == nullptr it only measures.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T> T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += sizeof(T) * std::max<size_t>(n, 1);
    return p;
  }
};

hipStream_t S(void* s) { return (hipStream_t)s; }

constexpr int kMaxTheta = 128;
constexpr int kTileItems = kTileSize;
constexpr int kRebuildMaxTiles = 128;

}  // namespace

struct mdvrp_instance {
  mdvrp_instance_desc d;
  int N = 0;
  int32_t* nbr = nullptr;
  int32_t* nbr_len = nullptr;
  int2* nbr_ct = nullptr;  // {c, t} of every list slot
  int4* attr = nullptr;
  int4* dep_arc = nullptr;  // depot-arc table (null beyond kDepArcMaxDepots depots)
  int64_t* partial = nullptr;
  int64_t* stats = nullptr;
  int nblocks = 0;
  int64_t Theta = 0, gnum = 1, gden = 1, w_depot = 0, max_c = 0, min_c = 0, max_t = 0;
  int64_t len_guard = 0;
  int t_is_c = 0;
  int64_t route_est = 1;                // routes a solution is expected to hold: 2 * ceil(sum q / Q)
  int32_t *cl = nullptr, *tl = nullptr, *pi = nullptr, *inv = nullptr, *corder = nullptr;  // locality layout
  int64_t* lm = nullptr;
  uint64_t* keys = nullptr;
  float frcp[4] = {1.f, 1.f, 1.f, 1.f};  // feature scales of the learned filter
};

// Scoring network: device buffers carved from the caller's workspace.
struct mdvrp_mlp {
  MlpDev d{};
};

// Opt-in per-launch timing with HIP events on the launch stream.
struct Profiler {
  bool on = false;
  uint32_t mask = 0;  // kernel classes timed
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;  // kernel class of pending event pair k
  int used = 0;
  int every = 1;            // time every n-th launch of a class
  int64_t seen[8] = {0};    // launches of each class since enabling (timed or not)
  int64_t launches[8] = {0};
  double ms[8] = {0};
  void reset() {
    used = 0;
    for (int k = 0; k < 8; ++k) { launches[k] = 0; ms[k] = 0; seen[k] = 0; }
  }
};

struct mdvrp_batch {
  Profiler prof;
  std::vector<const mdvrp_instance*> inst;
  std::vector<int> unit_inst;
  int n_units = 0;
  int has_tw = 0, open = 0;
  std::vector<UnitDesc> h_units;
  UnitDesc* d_units = nullptr;
  int32_t* d_tile_off[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<int32_t> h_tile_off[4];
  int32_t* d_active = nullptr;
  int32_t* d_act = nullptr;         // active map of the search's current pass (act_map_words)
  int32_t* d_node_base = nullptr;
  int32_t* d_route_base = nullptr;
  int64_t* d_state = nullptr;
  int64_t n_anchors = 0;            // sum over units of n_customers * theta
  int n_cust = 0;                   // sum over units of n_customers
  int kc = 0;                       // filtered list length (0 = no filter attached)
  int32_t* d_cust_off = nullptr;    // [n_units + 1] customer offsets (filter workspace)
  int32_t* d_tile_off_f = nullptr;  // [n_units + 1] filtered pair tiles (filter workspace)
  std::vector<int32_t> h_tile_off_f;
  int32_t* d_tile_off_r = nullptr;  // [n_units + 1] Depot-Replace compact grid (batch workspace)
  std::vector<int32_t> h_tile_off_r;
  FilterQueue stale{};              // stale-customer queue of the re-ranking (filter workspace)
  // captured passes of the local search, keyed by everything the launch sequence depends on
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
  hipStream_t own = nullptr;        // capture stream used when the caller passes the null stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // convergence poll of the search: active-unit counts of two poll intervals in pinned
  // host memory, each with the event that marks its copy
  int32_t* h_poll = nullptr;
  hipEvent_t ev_poll[2] = {nullptr, nullptr};
  // call order: the device state is defined only after a load; a selection needs an
  // evaluation of the same families on the current state, an apply needs a selection
  bool loaded = false;
  bool partial = false;    // loaded solutions miss customers (mdvrp_solutions_load_partial)
  int max_missing = 0;     // most customers missing from one unit's partial solution
  uint32_t eval_fam = 0;  // families of the latest evaluation of the current state (0 = none)
  bool planned = false;
  void state_changed() { eval_fam = 0; planned = false; }
  double clock_khz = 0;             // device wall-clock rate
  int shape[6] = {0, 0, 0, 0, 0, 0};  // tile shape of each family's evaluation (autotuner)
  // tile shape of an evaluation of fam_mask: the tuned one of a single family, else the default
  int shape_for(uint32_t fam_mask) const {
    for (int f = 0; f < 6; ++f)
      if (fam_mask == (1u << f)) return shape[f];
    return 0;
  }
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }
  // The passes of a search visit the active units' tiles only (active map written by
  // each pass's first kernel): the active units' tiles take the first blocks of every
  // launch, so that they are dispatched first and the blocks of converged units, which
  // have nothing to do, follow. Grids keep one block per tile of all units (one tile
  // per block lets the hardware balance the tiles' uneven costs).
  void search_grids(LaunchCtx& L) const { L.act = d_act; }
  LaunchCtx ctx(void* stream) const {
    bool layout_all = true;
    for (const mdvrp_instance* I : inst) layout_all = layout_all && I->pi != nullptr;
    LaunchCtx L;
    L.stream = S(stream);
    L.units = d_units;
    L.n_units = n_units;
    L.has_tw = has_tw;
    L.max_nd = 0;
    L.t_is_c_all = 1;
    for (const mdvrp_instance* I : inst) {
      L.max_nd = std::max(L.max_nd, I->d.n_depots);
      L.t_is_c_all = L.t_is_c_all && I->t_is_c;
    }
    L.open = open;
    for (int k = 0; k < 4; ++k) {
      L.tile_off[k] = d_tile_off[k];
      L.tiles[k] = h_tile_off[k].empty() ? 0 : h_tile_off[k].back();
      // unit-interleaved tile order: for instances kept in the locality layout (large
      // matrices), when every unit has the same tile count
      int per = n_units > 1 && layout_all && L.tiles[k] % n_units == 0 ? L.tiles[k] / n_units : 0;
      for (int u = 0; u < n_units && per > 0; ++u)
        if (h_tile_off[k][u + 1] - h_tile_off[k][u] != per) per = 0;
      L.per_unit[k] = per;
    }
    L.active_count = d_active;
    L.act = nullptr;
    L.adapt_units = nullptr;
    L.adapt = AdaptBounds{};
    auto per = [&](const std::vector<int32_t>& off) {
      if (off.size() != (size_t)n_units + 1 || n_units < 2 || !layout_all) return 0;
      const int p = off[1] - off[0];
      for (int u = 0; u < n_units; ++u)
        if (off[u + 1] - off[u] != p) return 0;
      return p;
    };
    L.tile_off_f = d_tile_off_f;
    L.tiles_f = h_tile_off_f.empty() ? 0 : h_tile_off_f.back();
    L.per_unit_f = per(h_tile_off_f);
    L.tile_off_r = d_tile_off_r;
    L.tiles_r = h_tile_off_r.empty() ? 0 : h_tile_off_r.back();
    L.per_unit_r = per(h_tile_off_r);
    L.compact = 0;
    return L;
  }
};

// ============================================================================ misc

extern "C" const char* mdvrp_status_string(mdvrp_status s) {
  switch (s) {
    case MDVRP_OK: return "ok";
    case MDVRP_EINVAL: return "invalid argument";
    case MDVRP_ERANGE: return "value out of the fixed-point range";
    case MDVRP_ENOSPC: return "insufficient space";
    case MDVRP_EDEVICE: return "device error";
    case MDVRP_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

extern "C" const char* mdvrp_last_error(void) { return g_err.c_str(); }

// Algorithm 2 visits the operator families in a random order each pass.
extern "C" int32_t mdvrp_family_order(int32_t has_tw, uint64_t seed, int64_t pass, int32_t* fam) {
  int n = 0;
  fam[n++] = FAM_REL;
  fam[n++] = FAM_SWP;
  fam[n++] = FAM_X2;
  if (!has_tw) fam[n++] = FAM_2OPT;
  fam[n++] = FAM_DINS;
  fam[n++] = FAM_DREP;
  uint64_t st = seed ^ (uint64_t)pass;
  for (int i = n - 1; i >= 1; --i) {
    const int j = (int)(splitmix64_next(&st) % (uint64_t)(i + 1));
    std::swap(fam[i], fam[j]);
  }
  return n;
}

// ============================================================================ instance

static mdvrp_status check_scalars(const mdvrp_instance_desc* d) {
  if (!d) return fail(MDVRP_EINVAL, "null descriptor");
  if (d->n_depots < 1 || d->n_customers < 1) return fail(MDVRP_EINVAL, "need at least one depot and one customer");
  if ((int64_t)d->n_depots + d->n_customers > 65535) return fail(MDVRP_EINVAL, "N = %d exceeds 65535",
                                                                  d->n_depots + d->n_customers);
  if (d->Q <= 0) return fail(MDVRP_EINVAL, "Q must be > 0");
  if (d->NV < 0) return fail(MDVRP_EINVAL, "NV must be >= 0");
  if (d->theta < 1 || d->theta > kMaxTheta) return fail(MDVRP_EINVAL, "theta must be in [1, %d]", kMaxTheta);
  if (d->w_tw < 0 || d->w_load < 0 || d->w_dur < 0) return fail(MDVRP_EINVAL, "penalty weights must be >= 0");
  if (d->open_routes != 0 && d->open_routes != 1) return fail(MDVRP_EINVAL, "open_routes must be 0 or 1");
  if (d->has_tw != 0 && d->has_tw != 1) return fail(MDVRP_EINVAL, "has_tw must be 0 or 1");
  if (d->layout < MDVRP_LAYOUT_AUTO || d->layout > MDVRP_LAYOUT_ORDERED) return fail(MDVRP_EINVAL, "unknown layout");
  if (!d->c || !d->t || !d->q || !d->s || !d->e || !d->l) return fail(MDVRP_EINVAL, "null array");
  return MDVRP_OK;
}

static mdvrp_status check_node_arrays(const mdvrp_instance_desc* d, const int32_t* q, const int32_t* s,
                                      const int32_t* e, const int32_t* l) {
  const int n = d->n_depots + d->n_customers;
  int64_t q_total = 0;
  for (int x = 0; x < n; ++x) {
    if (q[x] < 0 || s[x] < 0) return fail(MDVRP_EINVAL, "node %d: negative demand or service", x);
    q_total += q[x];
    if (e[x] > l[x]) return fail(MDVRP_EINVAL, "node %d: e > l", x);
    if (x < d->n_depots && (q[x] != 0 || s[x] != 0)) return fail(MDVRP_EINVAL, "depot %d: q and s must be 0", x);
  }
  // route loads (and the load deltas of a move) stay int32-safe
  if (q_total >= (1ll << 30)) return fail(MDVRP_ERANGE, "total demand %lld >= 2^30", (long long)q_total);
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_validate_instance_host(const mdvrp_instance_desc* d) {
  mdvrp_status st = check_scalars(d);
  if (st) return st;
  return check_node_arrays(d, d->q, d->s, d->e, d->l);
}

// Whether an instance keeps a locality-ordered copy of its matrices: asked for, or
// by default for matrices beyond what the caches hold.
static bool uses_layout(const mdvrp_instance_desc* d) {
  const int64_t n = (int64_t)d->n_depots + d->n_customers;
  if (d->layout == MDVRP_LAYOUT_GIVEN) return false;
  if (d->layout == MDVRP_LAYOUT_ORDERED) return true;
  return n * n * 4 > ((int64_t)64 << 20);
}

// Instances with at most this many depots keep a depot-arc table (16 bytes per
// customer and depot) for the depot operators; larger ones read the matrices.
constexpr int kDepArcMaxDepots = 64;

static void carve_instance(Carve& cv, const mdvrp_instance_desc* d, mdvrp_instance* I) {
  const int n = d->n_depots + d->n_customers;
  const int nb = inst_stats_blocks(n);
  int32_t* nbr = cv.take<int32_t>((size_t)d->n_customers * d->theta);
  int32_t* nbl = cv.take<int32_t>(d->n_customers);
  int2* nct = cv.take<int2>((size_t)d->n_customers * d->theta);
  int4* attr = cv.take<int4>(n);
  int4* dep_arc = d->n_depots <= kDepArcMaxDepots ? cv.take<int4>((size_t)d->n_customers * d->n_depots) : nullptr;
  int64_t* part = cv.take<int64_t>((size_t)nb * 8);
  int64_t* st = cv.take<int64_t>(8);
  if (I) {
    I->nbr = nbr;
    I->nbr_len = nbl;
    I->nbr_ct = nct;
    I->attr = attr;
    I->dep_arc = dep_arc;
    I->partial = part;
    I->stats = st;
    I->nblocks = nb;
  }
  if (uses_layout(d)) {
    int32_t* cl = cv.take<int32_t>((size_t)n * n);
    int32_t* tl = d->t != d->c ? cv.take<int32_t>((size_t)n * n) : nullptr;
    int32_t* pi = cv.take<int32_t>(n);
    int32_t* inv = cv.take<int32_t>(n);
    int32_t* co = cv.take<int32_t>(d->n_customers);
    int64_t* lm = cv.take<int64_t>(8);
    uint64_t* keys = cv.take<uint64_t>(n);
    if (I) {
      I->cl = cl; I->tl = tl; I->pi = pi; I->inv = inv; I->corder = co; I->lm = lm; I->keys = keys;
    }
  }
}

extern "C" mdvrp_status mdvrp_instance_workspace_query(const mdvrp_instance_desc* d, size_t* bytes) {
  mdvrp_status st = check_scalars(d);
  if (st) return st;
  if (!bytes) return fail(MDVRP_EINVAL, "null bytes");
  Carve cv(nullptr);
  carve_instance(cv, d, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

static int64_t gcd64(int64_t a, int64_t b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) { const int64_t r = a % b; a = b; b = r; }
  return a;
}

extern "C" mdvrp_status mdvrp_instance_create(const mdvrp_instance_desc* d, void* ws, size_t ws_bytes, void* stream,
                                              mdvrp_instance** out) {
  mdvrp_status st = check_scalars(d);
  if (st) return st;
  if (!out) return fail(MDVRP_EINVAL, "null out");
  size_t need = 0;
  mdvrp_instance_workspace_query(d, &need);
  if (!ws || ws_bytes < need) return fail(MDVRP_ENOSPC, "instance workspace needs %zu bytes", need);
  const int n = d->n_depots + d->n_customers;
  std::vector<int32_t> q(n), s(n), e(n), l(n);
  HIP_TRY(hipMemcpyAsync(q.data(), d->q, sizeof(int32_t) * n, hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemcpyAsync(s.data(), d->s, sizeof(int32_t) * n, hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemcpyAsync(e.data(), d->e, sizeof(int32_t) * n, hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemcpyAsync(l.data(), d->l, sizeof(int32_t) * n, hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  st = check_node_arrays(d, q.data(), s.data(), e.data(), l.data());
  if (st) return st;

  mdvrp_instance* I = new mdvrp_instance();
  I->d = *d;
  I->N = n;
  I->t_is_c = d->t == d->c;
  {
    int64_t sq = 0;
    for (int x = 0; x < n; ++x) sq += q[x];
    I->route_est = std::max<int64_t>(1, 2 * ((sq + d->Q - 1) / d->Q));
  }
  Carve cv(ws);
  carve_instance(cv, d, I);
  launch_node_attr(S(stream), d->q, d->s, d->e, d->l, n, I->attr);
  if (I->dep_arc) launch_depot_arcs(S(stream), d->c, d->t, d->n_depots, d->n_customers, I->dep_arc);
  launch_inst_stats(S(stream), d->c, d->t, n, I->partial, I->nblocks);
  launch_inst_stats_final(S(stream), I->partial, I->nblocks, I->stats);
  int64_t h[8];
  hipError_t he = hipMemcpyAsync(h, I->stats, sizeof h, hipMemcpyDeviceToHost, S(stream));
  if (he == hipSuccess) he = hipStreamSynchronize(S(stream));
  if (he != hipSuccess) {
    delete I;
    return fail(MDVRP_EDEVICE, "instance statistics: %s", hipGetErrorString(he));
  }
  if (h[5]) { delete I; return fail(MDVRP_EINVAL, "negative entries in c or t"); }
  if (!d->has_tw && h[4]) { delete I; return fail(MDVRP_EINVAL, "c/t must be symmetric without time windows"); }
  I->max_c = n > 1 ? h[0] : 0;
  I->min_c = n > 1 ? h[1] : 0;
  I->max_t = n > 1 ? h[6] : 0;
  I->Theta = 2 * I->max_c - I->min_c;
  const int64_t g = gcd64(h[2], h[3]);
  I->gnum = (h[3] == 0 || g == 0) ? 1 : h[2] / g;
  I->gden = (h[3] == 0 || g == 0) ? 1 : h[3] / g;
  I->w_depot = d->w_depot < 0 ? I->Theta : d->w_depot;
  // fixed-point guards
  if (8 * I->max_c >= (1ll << 25)) { delete I; return fail(MDVRP_ERANGE, "8*max c = %lld >= 2^25", (long long)(8 * I->max_c)); }
  int64_t smax = 0, emin = INT32_MAX, lmax = 0;
  for (int x = 0; x < n; ++x) {
    smax = std::max<int64_t>(smax, s[x]);
    emin = std::min<int64_t>(emin, e[x]);
    lmax = std::max<int64_t>(lmax, l[x]);
  }
  int64_t per_node = std::max<int64_t>(I->max_c, I->max_t + smax);
  if (d->has_tw) per_node = I->max_c + I->max_t + smax + (lmax - emin);
  I->len_guard = per_node > 0 ? ((int64_t)INT32_MAX / (2 * per_node)) - 2 : (int64_t)d->n_customers;
  if (I->len_guard < 2) { delete I; return fail(MDVRP_ERANGE, "values too large for int32 route segments"); }
  if (d->has_tw) {
    const __int128 span = (__int128)(lmax - emin) + smax + I->max_t;
    const __int128 kmax = (__int128)I->max_c * I->gden + (__int128)I->gnum * 11 * span;
    if (kmax >= ((__int128)1 << 62)) { delete I; return fail(MDVRP_ERANGE, "granular-list keys overflow int64"); }
  }
  launch_nbr_lists(S(stream), d->c, d->t, d->s, d->e, d->l, d->n_depots, d->n_customers, d->theta, d->has_tw,
                   I->gnum, I->gden, I->nbr, I->nbr_len);
  launch_nn_sum(S(stream), d->c, I->nbr, I->nbr_len, d->n_depots, d->n_customers, d->theta, I->stats);
  launch_nbr_arcs(S(stream), d->c, d->t, I->nbr, I->nbr_len, d->n_depots, d->n_customers, d->theta, I->nbr_ct);
  if (I->pi)
    launch_layout(S(stream), d->c, d->t, n, d->n_depots, I->lm, I->keys, I->pi, I->inv, I->corder, I->cl, I->tl);
  int64_t nn[2] = {0, 0};
  he = hipMemcpyAsync(nn, I->stats, sizeof nn, hipMemcpyDeviceToHost, S(stream));
  if (he == hipSuccess) he = hipStreamSynchronize(S(stream));
  if (he == hipSuccess) he = hipGetLastError();
  if (he != hipSuccess) {
    delete I;
    return fail(MDVRP_EDEVICE, "granular lists: %s", hipGetErrorString(he));
  }
  // filter feature scales: mean distance to the first list entry (integer mean, at
  // least 1), capacity, the time horizon of depot 0 (time windows only), depot count
  const int64_t dscale = std::max<int64_t>(1, nn[1] ? nn[0] / nn[1] : 1);
  const int64_t hscale = std::max<int64_t>(1, d->has_tw ? (int64_t)l[0] - e[0] : 1);
  I->frcp[0] = 1.0f / (float)dscale;
  I->frcp[1] = 1.0f / (float)d->Q;
  I->frcp[2] = 1.0f / (float)hscale;
  I->frcp[3] = 1.0f / (float)d->n_depots;
  *out = I;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_instance_info(const mdvrp_instance* I, int64_t out[8]) {
  if (!I || !out) return fail(MDVRP_EINVAL, "null argument");
  out[0] = I->Theta; out[1] = I->gnum; out[2] = I->gden; out[3] = I->w_depot;
  out[4] = I->max_c; out[5] = I->min_c; out[6] = I->max_t; out[7] = I->len_guard;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_instance_copy_lists(const mdvrp_instance* I, int32_t* nbr, int32_t* len, void* stream) {
  if (!I || !nbr || !len) return fail(MDVRP_EINVAL, "null argument");
  HIP_TRY(hipMemcpyAsync(nbr, I->nbr, sizeof(int32_t) * (size_t)I->d.n_customers * I->d.theta,
                         hipMemcpyDeviceToDevice, S(stream)));
  HIP_TRY(hipMemcpyAsync(len, I->nbr_len, sizeof(int32_t) * I->d.n_customers, hipMemcpyDeviceToDevice, S(stream)));
  return MDVRP_OK;
}

extern "C" void mdvrp_instance_destroy(mdvrp_instance* I) { delete I; }

// ============================================================================ batch

namespace {

struct UnitSizes {
  int nd, nc, n, R, cap, theta;
  int64_t cand_cap;
  int tiles[4];
};

UnitSizes unit_sizes(const mdvrp_instance* I) {
  UnitSizes z;
  z.nd = I->d.n_depots;
  z.nc = I->d.n_customers;
  z.n = z.nd + z.nc;
  z.R = z.nc;
  // positions of one buffer: a solution takes n_customers + 2 M <= 3 n_customers of them;
  // the rest is room for rebuilt routes appended in place between relayouts
  z.cap = 6 * z.nc + 256;
  z.theta = I->d.theta;
  z.cand_cap = 3ll * z.nc * z.theta + 2ll * z.nc * z.nd + 64;
  z.tiles[0] = (int)(((int64_t)z.nc * z.theta + kTileItems - 1) / kTileItems);
  z.tiles[1] = (int)(((int64_t)z.nc * z.nd + kTileItems - 1) / kTileItems);
  z.tiles[2] = z.tiles[1];
  // rebuild blocks (4 wavefronts, one route each, grid-stride over the alive routes):
  // enough for the routes a solution is expected to hold
  z.tiles[3] = (int)std::max<int64_t>(1, std::min<int64_t>({kRebuildMaxTiles, (z.R + 3) / 4, (I->route_est + 3) / 4}));
  return z;
}

// Per-unit device state; with base == nullptr only the size is measured.
void carve_unit(Carve& cv, const mdvrp_instance* I, int has_tw, UnitDesc* U) {
  const UnitSizes z = unit_sizes(I);
  const size_t seg = has_tw ? sizeof(SegTW) : sizeof(SegNT);
  UnitDesc u{};
  u.rt = cv.take<int32_t>(z.n);
  u.pos = cv.take<int32_t>(z.n);
  u.apos = cv.take<int32_t>(z.n);
  u.r_len = cv.take<int32_t>(z.R);
  u.r_start = cv.take<int32_t>(z.R);
  u.r_end = cv.take<int32_t>(z.R);
  u.r_off[0] = cv.take<int32_t>(z.R);
  u.r_off[1] = cv.take<int32_t>(z.R);
  u.r_meta[0] = cv.take<int4>(z.R);
  u.r_meta[1] = cv.take<int4>(z.R);
  u.r_tot = cv.take<int4>(z.R);
  u.r_core = has_tw ? cv.take<SegTW>(z.R) : nullptr;
  for (int b = 0; b < 2; ++b) {
    u.fw[b] = cv.take<char>(seg * z.cap);
    u.bw[b] = cv.take<char>(seg * z.cap);
  }
  u.ndep = cv.take<int32_t>(z.nd);
  u.ctl = cv.take<UnitCtl>(1);
  u.cand_key = cv.take<uint64_t>(z.cand_cap);
  u.cand_id = cv.take<uint64_t>(z.cand_cap);
  u.cand_res = cv.take<int4>(z.cand_cap);
  u.cand_alive = cv.take<uint8_t>(z.cand_cap);
  u.resmin = cv.take<uint64_t>(z.R + z.nd);
  u.taken = cv.take<int32_t>(z.R + z.nd);
  u.dirty = cv.take<int32_t>(z.R);
  u.plan_n = cv.take<int32_t>(z.R);
  u.plan_pc = cv.take<int4>((size_t)z.R * kMaxPieces);
  u.slot_list = cv.take<int32_t>(z.R);
  u.sel_size = cv.take<int32_t>(z.R + 1);
  u.sel_slot = cv.take<int32_t>(2 * ((size_t)z.R + 1));
  u.build_list = cv.take<int32_t>(z.R);
  u.sel_id = cv.take<uint64_t>(z.R + 1);
  u.sel_dF = cv.take<int64_t>(z.R + 1);
  u.wg_best = cv.take<MoveRec>((size_t)z.tiles[0] + z.tiles[1] + z.tiles[2]);
  if (U) *U = u;
}

mdvrp_status check_batch_args(const mdvrp_instance* const* insts, int32_t n_inst, const int32_t* unit_inst,
                              int32_t n_units) {
  if (!insts || n_inst < 1 || !unit_inst || n_units < 1) return fail(MDVRP_EINVAL, "empty batch");
  for (int k = 0; k < n_inst; ++k)
    if (!insts[k]) return fail(MDVRP_EINVAL, "null instance %d", k);
  for (int k = 0; k < n_units; ++k)
    if (unit_inst[k] < 0 || unit_inst[k] >= n_inst) return fail(MDVRP_EINVAL, "unit %d: bad instance index", k);
  for (int k = 1; k < n_inst; ++k)
    if (insts[k]->d.has_tw != insts[0]->d.has_tw || insts[k]->d.open_routes != insts[0]->d.open_routes)
      return fail(MDVRP_EINVAL, "instances of a batch must agree on has_tw and open_routes");
  return MDVRP_OK;
}

void carve_batch(Carve& cv, const mdvrp_instance* const* insts, const int32_t* unit_inst, int32_t n_units,
                 mdvrp_batch* B) {
  const int has_tw = insts[0]->d.has_tw;
  UnitDesc* du = cv.take<UnitDesc>(n_units);
  int32_t* to[4];
  for (int k = 0; k < 4; ++k) to[k] = cv.take<int32_t>(n_units + 1);
  int32_t* tor = cv.take<int32_t>(n_units + 1);
  int32_t* act = cv.take<int32_t>(1);
  int32_t* amap = cv.take<int32_t>((size_t)act_map_words(n_units));
  int32_t* nb = cv.take<int32_t>(n_units);
  int32_t* rb = cv.take<int32_t>(n_units);
  int64_t* stt = cv.take<int64_t>((size_t)n_units * kStateWords);
  if (B) {
    B->d_units = du;
    for (int k = 0; k < 4; ++k) B->d_tile_off[k] = to[k];
    B->d_tile_off_r = tor;
    B->d_active = act;
    B->d_act = amap;
    B->d_node_base = nb;
    B->d_route_base = rb;
    B->d_state = stt;
    B->h_units.resize(n_units);
  }
  for (int k = 0; k < n_units; ++k) carve_unit(cv, insts[unit_inst[k]], has_tw, B ? &B->h_units[k] : nullptr);
}

}  // namespace

extern "C" mdvrp_status mdvrp_batch_workspace_query(const mdvrp_instance* const* insts, int32_t n_inst,
                                                    const int32_t* unit_inst, int32_t n_units, size_t* bytes) {
  mdvrp_status st = check_batch_args(insts, n_inst, unit_inst, n_units);
  if (st) return st;
  if (!bytes) return fail(MDVRP_EINVAL, "null bytes");
  Carve cv(nullptr);
  carve_batch(cv, insts, unit_inst, n_units, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_batch_create(const mdvrp_instance* const* insts, int32_t n_inst,
                                           const int32_t* unit_inst, int32_t n_units, void* ws, size_t ws_bytes,
                                           void* stream, mdvrp_batch** out) {
  mdvrp_status st = check_batch_args(insts, n_inst, unit_inst, n_units);
  if (st) return st;
  if (!out) return fail(MDVRP_EINVAL, "null out");
  size_t need = 0;
  mdvrp_batch_workspace_query(insts, n_inst, unit_inst, n_units, &need);
  if (!ws || ws_bytes < need) return fail(MDVRP_ENOSPC, "batch workspace needs %zu bytes", need);
  mdvrp_batch* B = new mdvrp_batch();
  B->inst.assign(insts, insts + n_inst);
  B->unit_inst.assign(unit_inst, unit_inst + n_units);
  B->n_units = n_units;
  B->has_tw = insts[0]->d.has_tw;
  B->open = insts[0]->d.open_routes;
  Carve cv(ws);
  carve_batch(cv, insts, unit_inst, n_units, B);
  for (int k = 0; k < 4; ++k) B->h_tile_off[k].assign(1, 0);
  B->h_tile_off_r.assign(1, 0);
  std::vector<int32_t> nbase(n_units), rbase(n_units);
  int32_t nacc = 0, racc = 0;
  for (int k = 0; k < n_units; ++k) {
    const mdvrp_instance* I = insts[unit_inst[k]];
    const UnitSizes z = unit_sizes(I);
    UnitDesc& u = B->h_units[k];
    u.c = I->d.c; u.t = I->d.t; u.q = I->d.q; u.s = I->d.s; u.e = I->d.e; u.l = I->d.l;
    u.nbr = I->nbr; u.nbr_len = I->nbr_len; u.nbr_ct = I->nbr_ct; u.attr = I->attr; u.dep_arc = I->dep_arc;
    u.cl = I->cl; u.tl = I->tl ? I->tl : I->cl; u.pi = I->pi; u.corder = I->corder;
    u.nd = z.nd; u.nc = z.nc; u.n = z.n; u.theta = z.theta;
    u.Q = I->d.Q; u.NV = I->d.NV; u.Dmax = I->d.Dmax;
    u.w_tw = I->d.w_tw; u.w_load = I->d.w_load; u.w_dur = I->d.w_dur;
    u.w_depot = I->w_depot;
    u.R = z.R; u.cap = z.cap; u.t_is_c = I->t_is_c;
    u.cand_cap = (int32_t)std::min<int64_t>(z.cand_cap, INT32_MAX);
    u.len_guard = (int32_t)std::min<int64_t>(I->len_guard, INT32_MAX);
    u.tile_base[0] = 0;
    u.tile_base[1] = z.tiles[0];
    u.tile_base[2] = z.tiles[0] + z.tiles[1];
    u.tile_base[3] = z.tiles[0] + z.tiles[1] + z.tiles[2];
    u.key_shift = 38;
    u.item_base = B->n_anchors;
    B->n_anchors += (int64_t)z.nc * z.theta;
    B->n_cust += z.nc;
    for (int f = 0; f < 4; ++f) u.frcp[f] = I->frcp[f];
    for (int c = 0; c < 4; ++c) B->h_tile_off[c].push_back(B->h_tile_off[c].back() + z.tiles[c]);
    // Depot-Replace blocks for the routes a solution is expected to hold (a block loops
    // over more tiles when there are more routes)
    const int64_t rt = (I->route_est * z.nd + kTileItems - 1) / kTileItems;
    B->h_tile_off_r.push_back(B->h_tile_off_r.back() + (int32_t)std::max<int64_t>(1, std::min<int64_t>(rt, z.tiles[2])));
    nbase[k] = nacc;
    rbase[k] = racc;
    nacc += z.nc;
    racc += z.nc + 1;
  }
  hipStream_t s = S(stream);
  hipError_t he = hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * n_units, hipMemcpyHostToDevice, s);
  for (int c = 0; c < 4 && he == hipSuccess; ++c)
    he = hipMemcpyAsync(B->d_tile_off[c], B->h_tile_off[c].data(), sizeof(int32_t) * (n_units + 1),
                        hipMemcpyHostToDevice, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(B->d_tile_off_r, B->h_tile_off_r.data(), sizeof(int32_t) * (n_units + 1),
                        hipMemcpyHostToDevice, s);
  if (he == hipSuccess) {
    int dev = 0, khz = 0;
    he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    B->clock_khz = khz;
  }
  if (he == hipSuccess) he = hipMemcpyAsync(B->d_node_base, nbase.data(), sizeof(int32_t) * n_units, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(B->d_route_base, rbase.data(), sizeof(int32_t) * n_units, hipMemcpyHostToDevice, s);
  for (int k = 0; k < n_units && he == hipSuccess; ++k) {
    const UnitDesc& u = B->h_units[k];
    he = hipMemsetAsync(u.ctl, 0, sizeof(UnitCtl), s);
    if (he == hipSuccess) he = hipMemsetAsync(u.taken, 0, sizeof(int32_t) * (u.R + u.nd), s);
    if (he == hipSuccess) he = hipMemsetAsync(u.dirty, 0, sizeof(int32_t) * u.R, s);
    if (he == hipSuccess) he = hipMemsetAsync(u.r_len, 0, sizeof(int32_t) * u.R, s);
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    delete B;
    return fail(MDVRP_EDEVICE, "batch create: %s", hipGetErrorString(he));
  }
  *out = B;
  return MDVRP_OK;
}

extern "C" void mdvrp_batch_destroy(mdvrp_batch* B) {
  if (!B) return;
  for (hipEvent_t e : B->prof.ev) (void)hipEventDestroy(e);
  B->drop_graphs();
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  for (hipEvent_t e : B->ev_poll)
    if (e) (void)hipEventDestroy(e);
  if (B->h_poll) (void)hipHostFree(B->h_poll);
  if (B->own) (void)hipStreamDestroy(B->own);
  delete B;
}

// ============================================================================ profiling

extern "C" mdvrp_status mdvrp_profile_enable(mdvrp_batch* B, uint32_t class_mask, int32_t max_launches) {
  if (!B || max_launches < 0) return fail(MDVRP_EINVAL, "bad argument");
  Profiler& P = B->prof;
  P.reset();
  P.on = class_mask != 0;
  P.mask = class_mask;
  if (!P.on) return MDVRP_OK;
  const size_t need = 2 * (size_t)std::max(max_launches, 1);
  while (P.ev.size() < need) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    P.ev.push_back(e);
  }
  P.cls.assign(need / 2, 0);
  return MDVRP_OK;
}

// Resolve pending event pairs into per-class totals (synchronises the events).
static mdvrp_status profile_flush(Profiler& P) {
  for (int k = 0; k < P.used; ++k) {
    HIP_TRY(hipEventSynchronize(P.ev[2 * k + 1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, P.ev[2 * k], P.ev[2 * k + 1]));
    P.launches[P.cls[k]] += 1;
    P.ms[P.cls[k]] += t;
  }
  P.used = 0;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_profile_sampling(mdvrp_batch* B, int32_t every) {
  if (!B || every < 1) return fail(MDVRP_EINVAL, "bad argument");
  B->prof.every = every;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_profile_read(mdvrp_batch* B, int64_t* launches, double* ms) {
  if (!B || !launches || !ms) return fail(MDVRP_EINVAL, "null argument");
  mdvrp_status s = profile_flush(B->prof);
  if (s) return s;
  for (int k = 0; k < 8; ++k) { launches[k] = B->prof.launches[k]; ms[k] = B->prof.ms[k]; }
  return MDVRP_OK;
}

namespace {
// Launch one kernel class, bracketed by events when profiling is on.
template <class F>
void timed(mdvrp_batch* B, hipStream_t s, int cls, F&& launch) {
  Profiler& P = B->prof;
  if (!P.on || !(P.mask >> cls & 1)) { launch(); return; }
  if (P.seen[cls]++ % P.every != 0) { launch(); return; }
  if (P.used * 2 + 2 > (int)P.ev.size()) profile_flush(P);
  if (P.used * 2 + 2 > (int)P.ev.size()) { launch(); return; }
  const int k = P.used++;
  P.cls[k] = cls;
  (void)hipEventRecord(P.ev[2 * k], s);
  launch();
  (void)hipEventRecord(P.ev[2 * k + 1], s);
}
}  // namespace

// Solutions loaded, possibly partial (customers missing).
static mdvrp_status need_loaded_any(const mdvrp_batch* B) {
  return B->loaded ? MDVRP_OK : fail(MDVRP_ESTATE, "no solutions loaded in this batch");
}

// Complete solutions loaded (every customer routed): what the evaluation, selection,
// search, filter and population calls need.
static mdvrp_status need_loaded(const mdvrp_batch* B) {
  if (mdvrp_status e = need_loaded_any(B)) return e;
  return B->partial ? fail(MDVRP_ESTATE, "the batch holds partial solutions: call mdvrp_repair first") : MDVRP_OK;
}

// Checks of mdvrp_validate_solutions_host; with missing != nullptr customers may be
// absent (partial solutions) and missing[k] receives unit k's count of them.
static mdvrp_status validate_solutions(const mdvrp_instance_desc* descs, int32_t n_inst, const int32_t* unit_inst,
                                       int32_t n_units, const int32_t* nodes, const int32_t* offs,
                                       const int32_t* starts, const int32_t* ends, const int32_t* uro,
                                       std::vector<int>* missing);

extern "C" mdvrp_status mdvrp_validate_solutions_host(const mdvrp_instance_desc* descs, int32_t n_inst,
                                                      const int32_t* unit_inst, int32_t n_units, const int32_t* nodes,
                                                      const int32_t* offs, const int32_t* starts, const int32_t* ends,
                                                      const int32_t* uro) {
  return validate_solutions(descs, n_inst, unit_inst, n_units, nodes, offs, starts, ends, uro, nullptr);
}

static mdvrp_status validate_solutions(const mdvrp_instance_desc* descs, int32_t n_inst, const int32_t* unit_inst,
                                       int32_t n_units, const int32_t* nodes, const int32_t* offs,
                                       const int32_t* starts, const int32_t* ends, const int32_t* uro,
                                       std::vector<int>* missing) {
  if (!descs || !unit_inst || !nodes || !offs || !starts || !ends || !uro || n_inst < 1 || n_units < 1)
    return fail(MDVRP_EINVAL, "null argument");
  std::vector<int32_t> seen;
  for (int k = 0; k < n_units; ++k) {
    if (unit_inst[k] < 0 || unit_inst[k] >= n_inst) return fail(MDVRP_EINVAL, "unit %d: bad instance index", k);
    const mdvrp_instance_desc& D = descs[unit_inst[k]];
    const int nd = D.n_depots, nc = D.n_customers, n = nd + nc;
    const int r0 = uro[k], r1 = uro[k + 1];
    if (r1 < r0) return fail(MDVRP_EINVAL, "unit %d: decreasing route offsets", k);
    if (r1 - r0 > nc) return fail(MDVRP_EINVAL, "unit %d: more routes than customers", k);
    seen.assign(n, 0);
    int count = 0;
    for (int r = r0; r < r1; ++r) {
      const int a = offs[r], b = offs[r + 1];
      if (b <= a) return fail(MDVRP_EINVAL, "unit %d route %d: empty route", k, r - r0);
      if (starts[r] < 0 || starts[r] >= nd) return fail(MDVRP_EINVAL, "unit %d route %d: start is not a depot", k, r - r0);
      if (!D.open_routes && (ends[r] < 0 || ends[r] >= nd))
        return fail(MDVRP_EINVAL, "unit %d route %d: end is not a depot", k, r - r0);
      for (int p = a; p < b; ++p) {
        const int x = nodes[p];
        if (x < nd || x >= n) return fail(MDVRP_EINVAL, "unit %d: node %d is not a customer", k, x);
        if (seen[x]++) return fail(MDVRP_EINVAL, "unit %d: customer %d visited twice", k, x);
        ++count;
      }
    }
    if (missing) (*missing)[k] = nc - count;
    else if (count != nc) return fail(MDVRP_EINVAL, "unit %d: %d of %d customers routed", k, count, nc);
  }
  return MDVRP_OK;
}

// Reset every unit's penalty weights (host copy of the unit descriptors) to its
// instance's; true when any changed, so that the device copy needs an upload.
static bool weights_to_instance(mdvrp_batch* B) {
  bool changed = false;
  for (int k = 0; k < B->n_units; ++k) {
    const mdvrp_instance* I = B->inst[B->unit_inst[k]];
    UnitDesc& u = B->h_units[k];
    if (u.w_tw != I->d.w_tw || u.w_load != I->d.w_load || u.w_dur != I->d.w_dur || u.w_depot != I->w_depot) {
      u.w_tw = I->d.w_tw;
      u.w_load = I->d.w_load;
      u.w_dur = I->d.w_dur;
      u.w_depot = I->w_depot;
      changed = true;
    }
  }
  return changed;
}

// Solutions of every unit from device arrays; partial = customers may be missing.
static mdvrp_status load_solutions(mdvrp_batch* B, const int32_t* nodes, const int32_t* offs, const int32_t* starts,
                                   const int32_t* ends, const int32_t* uro, int32_t n_routes, int32_t n_nodes,
                                   void* stream, bool partial) {
  if (!B || !nodes || !offs || !starts || !ends || !uro) return fail(MDVRP_EINVAL, "null argument");
  if (n_routes < 0 || n_nodes < 0) return fail(MDVRP_EINVAL, "negative sizes");
  hipStream_t s = S(stream);
  std::vector<int32_t> hn(std::max(n_nodes, 1)), ho(n_routes + 1), hs(std::max(n_routes, 1)),
      he_(std::max(n_routes, 1)), hu(B->n_units + 1);
  HIP_TRY(hipMemcpyAsync(hu.data(), uro, sizeof(int32_t) * (B->n_units + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ho.data(), offs, sizeof(int32_t) * (n_routes + 1), hipMemcpyDeviceToHost, s));
  if (n_nodes) HIP_TRY(hipMemcpyAsync(hn.data(), nodes, sizeof(int32_t) * n_nodes, hipMemcpyDeviceToHost, s));
  if (n_routes) {
    HIP_TRY(hipMemcpyAsync(hs.data(), starts, sizeof(int32_t) * n_routes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(he_.data(), ends, sizeof(int32_t) * n_routes, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (hu[0] != 0 || hu[B->n_units] != n_routes) return fail(MDVRP_EINVAL, "unit route offsets do not span the routes");
  if (ho[0] != 0 || ho[n_routes] != n_nodes) return fail(MDVRP_EINVAL, "route offsets do not span the nodes");
  for (int r = 0; r < n_routes; ++r)
    if (ho[r + 1] < ho[r]) return fail(MDVRP_EINVAL, "decreasing route offsets");
  std::vector<mdvrp_instance_desc> descs;
  for (const mdvrp_instance* I : B->inst) descs.push_back(I->d);
  std::vector<int> missing(B->n_units, 0);
  mdvrp_status st = validate_solutions(descs.data(), (int32_t)descs.size(), B->unit_inst.data(), B->n_units,
                                       hn.data(), ho.data(), hs.data(), he_.data(), hu.data(),
                                       partial ? &missing : nullptr);
  if (st) return st;
  // the segment arithmetic is int32: a route longer than the instance's guard could overflow
  // (a partial solution: not even when every missing customer joins its longest route)
  int max_missing = 0;
  for (int k = 0; k < B->n_units; ++k) {
    const int64_t guard = B->inst[B->unit_inst[k]]->len_guard;
    for (int r = hu[k]; r < hu[k + 1]; ++r)
      if (ho[r + 1] - ho[r] + missing[k] > guard)
        return fail(MDVRP_ERANGE, "unit %d route %d: %d customers (and %d missing), beyond the int32-safe length %lld",
                    k, r - hu[k], ho[r + 1] - ho[r], missing[k], (long long)guard);
    if (missing[k] > guard) return fail(MDVRP_ERANGE, "unit %d: %d missing customers, beyond the int32-safe length",
                                        k, missing[k]);
    max_missing = std::max(max_missing, missing[k]);
  }
  const LaunchCtx L = B->ctx(stream);
  B->loaded = false;
  B->state_changed();
  if (weights_to_instance(B))
    HIP_TRY(hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
  launch_load(L, nodes, offs, starts, ends, uro);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  B->loaded = true;
  B->partial = partial && max_missing > 0;
  B->max_missing = partial ? max_missing : 0;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_solutions_load(mdvrp_batch* B, const int32_t* nodes, const int32_t* offs,
                                             const int32_t* starts, const int32_t* ends, const int32_t* uro,
                                             int32_t n_routes, int32_t n_nodes, void* stream) {
  return load_solutions(B, nodes, offs, starts, ends, uro, n_routes, n_nodes, stream, false);
}

extern "C" mdvrp_status mdvrp_solutions_load_partial(mdvrp_batch* B, const int32_t* nodes, const int32_t* offs,
                                                     const int32_t* starts, const int32_t* ends, const int32_t* uro,
                                                     int32_t n_routes, int32_t n_nodes, void* stream) {
  return load_solutions(B, nodes, offs, starts, ends, uro, n_routes, n_nodes, stream, true);
}

static mdvrp_status check_unit_errors(mdvrp_batch* B, std::vector<int64_t>& st, void* stream);

extern "C" mdvrp_status mdvrp_repair(mdvrp_batch* B, int32_t op, uint64_t seed, int32_t* order, int64_t* n_evaluated,
                                     void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  if (op < MDVRP_REPAIR_FBI || op > MDVRP_REPAIR_RI) return fail(MDVRP_EINVAL, "unknown insertion operator %d", op);
  if (mdvrp_status e = need_loaded_any(B)) return e;
  B->state_changed();
  const LaunchCtx L = B->ctx(stream);
  launch_ins_begin(L);
  for (int r = 0; r < B->max_missing; ++r) launch_ins_round(L, op, seed, B->max_missing, order, B->d_node_base);
  HIP_TRY(hipGetLastError());
  launch_cost(L, nullptr, nullptr);
  if (n_evaluated) launch_ins_export(L, n_evaluated);
  std::vector<int64_t> stv;
  mdvrp_status s = check_unit_errors(B, stv, stream);
  if (s) return s;
  B->partial = false;
  B->max_missing = 0;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_solutions_export(const mdvrp_batch* B, int32_t* nodes, int32_t* offs, int32_t* starts,
                                               int32_t* ends, int32_t* counts, void* stream) {
  if (!B || !nodes || !offs || !starts || !ends || !counts) return fail(MDVRP_EINVAL, "null argument");
  if (mdvrp_status e = need_loaded_any(B)) return e;
  const LaunchCtx L = B->ctx(stream);
  launch_export(L, nodes, offs, starts, ends, counts, B->d_node_base, B->d_route_base);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_batch_cost(mdvrp_batch* B, int64_t* F, int64_t* terms, void* stream) {
  if (!B || !F) return fail(MDVRP_EINVAL, "null argument");
  if (mdvrp_status e = need_loaded_any(B)) return e;
  launch_cost(B->ctx(stream), F, terms);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

// ============================================================================ population (Section 3.4)

namespace {

// Workspace of a population call: the member list and the per-member edge keys and
// edge counts.
void carve_pop(Carve& cv, int n, int nc, int32_t** list, int2** keys, int64_t** n_edges) {
  int32_t* l = cv.take<int32_t>(n);
  int2* k = cv.take<int2>((size_t)n * nc);
  int64_t* e = cv.take<int64_t>(n);
  if (list) *list = l;
  if (keys) *keys = k;
  if (n_edges) *n_edges = e;
}

// Members: distinct units of the batch, all of one instance.
mdvrp_status check_members(const mdvrp_batch* B, const int32_t* units, int32_t n, int* nc) {
  if (!B || !units || n < 1 || n > kPopMaxMembers)
    return fail(MDVRP_EINVAL, "population of %d members (1..%d)", n, kPopMaxMembers);
  std::vector<char> seen(B->n_units, 0);
  for (int i = 0; i < n; ++i) {
    const int u = units[i];
    if (u < 0 || u >= B->n_units) return fail(MDVRP_EINVAL, "member %d: unit %d out of range", i, u);
    if (seen[u]) return fail(MDVRP_EINVAL, "member %d: unit %d listed twice", i, u);
    seen[u] = 1;
    if (B->unit_inst[u] != B->unit_inst[units[0]])
      return fail(MDVRP_EINVAL, "member %d: unit %d belongs to another instance", i, u);
  }
  *nc = B->h_units[units[0]].nc;
  return MDVRP_OK;
}

}  // namespace

extern "C" mdvrp_status mdvrp_population_workspace_query(const mdvrp_batch* B, const int32_t* units, int32_t n,
                                                         size_t* bytes) {
  if (!bytes) return fail(MDVRP_EINVAL, "null bytes");
  int nc = 0;
  if (mdvrp_status e = check_members(B, units, n, &nc)) return e;
  Carve cv(nullptr);
  carve_pop(cv, n, nc, nullptr, nullptr, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_population_distance(mdvrp_batch* B, const int32_t* units, int32_t n, double* dist,
                                                  int64_t* common, int64_t* n_edges, void* ws, size_t ws_bytes,
                                                  void* stream) {
  int nc = 0;
  if (mdvrp_status e = check_members(B, units, n, &nc)) return e;
  if (!dist) return fail(MDVRP_EINVAL, "null dist");
  if (mdvrp_status e = need_loaded(B)) return e;
  Carve need(nullptr);
  carve_pop(need, n, nc, nullptr, nullptr, nullptr);
  if (!ws || ws_bytes < need.off + 256) return fail(MDVRP_ENOSPC, "population workspace needs %zu bytes", need.off + 256);
  Carve cv(ws);
  int32_t* list = nullptr;
  int2* keys = nullptr;
  int64_t* ne = nullptr;
  carve_pop(cv, n, nc, &list, &keys, &ne);
  const LaunchCtx L = B->ctx(stream);
  HIP_TRY(hipMemcpyAsync(list, units, sizeof(int32_t) * n, hipMemcpyHostToDevice, L.stream));
  launch_pop_distance(L, list, n, nc, keys, ne, dist, common);
  if (n_edges) HIP_TRY(hipMemcpyAsync(n_edges, ne, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, L.stream));
  HIP_TRY(hipGetLastError());
  // the member list was copied from the caller's host array: wait before returning
  HIP_TRY(hipStreamSynchronize(L.stream));
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_population_reduce(const double* dist, const int64_t* f, int32_t n, int32_t mu,
                                                double xi, int32_t n_close, int32_t* keep, int32_t* order,
                                                double* chi, double* dpop, void* stream) {
  if (!dist || !f || !keep) return fail(MDVRP_EINVAL, "null argument");
  if (n < 1 || n > kPopMaxMembers) return fail(MDVRP_EINVAL, "population of %d members (1..%d)", n, kPopMaxMembers);
  if (mu < 1) return fail(MDVRP_EINVAL, "mu must be >= 1");
  if (n_close < 1 || n_close > kPopMaxClose) return fail(MDVRP_EINVAL, "n_close must be 1..%d", kPopMaxClose);
  if (!(xi >= 0.0) || !(xi <= 1e6)) return fail(MDVRP_EINVAL, "xi must be a finite value >= 0");
  launch_pop_reduce(S(stream), dist, f, n, mu, xi, n_close, keep, order, chi, dpop);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

// ============================================================================ DCREX crossover (Algorithm 3, Eq. 4)

namespace {

// Host copy and checks of route lists given in device arrays: offsets from 0 to len,
// non-decreasing; customers in [nd, n); starts depots; ends depots or -1; flags 0/1;
// no customer twice in one route (unique_all: in the whole list).
mdvrp_status check_routes_dev(const char* what, int nd, int n, int nr, int len, const int32_t* nodes,
                              const int32_t* offs, const int32_t* start, const int32_t* end, const int32_t* flags,
                              bool unique_all, hipStream_t s) {
  if (nr < 0 || len < 0) return fail(MDVRP_EINVAL, "%s: negative sizes", what);
  if (nr == 0) return MDVRP_OK;
  if (!nodes || !offs || !start || !end) return fail(MDVRP_EINVAL, "%s: null array", what);
  std::vector<int32_t> hn(std::max(len, 1)), ho(nr + 1), hs(nr), he(nr), hf(flags ? nr : 0);
  HIP_TRY(hipMemcpyAsync(ho.data(), offs, sizeof(int32_t) * (nr + 1), hipMemcpyDeviceToHost, s));
  if (len) HIP_TRY(hipMemcpyAsync(hn.data(), nodes, sizeof(int32_t) * len, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hs.data(), start, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(he.data(), end, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
  if (flags) HIP_TRY(hipMemcpyAsync(hf.data(), flags, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ho[0] != 0 || ho[nr] != len) return fail(MDVRP_EINVAL, "%s: offsets do not span the nodes", what);
  std::vector<int32_t> seen(n, -1);
  for (int r = 0; r < nr; ++r) {
    if (ho[r + 1] < ho[r]) return fail(MDVRP_EINVAL, "%s: decreasing offsets", what);
    if (hs[r] < 0 || hs[r] >= nd) return fail(MDVRP_EINVAL, "%s route %d: start is not a depot", what, r);
    if (he[r] < -1 || he[r] >= nd) return fail(MDVRP_EINVAL, "%s route %d: end is neither a depot nor -1", what, r);
    if (flags && hf[r] != 0 && hf[r] != 1) return fail(MDVRP_EINVAL, "%s route %d: flag not 0 or 1", what, r);
    for (int p = ho[r]; p < ho[r + 1]; ++p) {
      const int x = hn[p];
      if (x < nd || x >= n) return fail(MDVRP_EINVAL, "%s route %d: node %d is not a customer", what, r, x);
      if (seen[x] == r || (unique_all && seen[x] >= 0))
        return fail(MDVRP_EINVAL, "%s: customer %d visited twice", what, x);
      seen[x] = r;
    }
  }
  return MDVRP_OK;
}

}  // namespace

extern "C" mdvrp_status mdvrp_dcrex_workspace_query(int32_t n_nodes, int32_t ns, int32_t np, int32_t p_len,
                                                    size_t* bytes) {
  if (!bytes || n_nodes < 1 || ns < 0 || np < 0 || p_len < 0) return fail(MDVRP_EINVAL, "bad argument");
  *bytes = dcrex_ws_bytes(n_nodes, ns, np, p_len) + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_dcrex_counts(int32_t n_depots, int32_t n_nodes, int32_t ns, int32_t s_len,
                                           const int32_t* s_nodes, const int32_t* s_offs, const int32_t* s_start,
                                           const int32_t* s_end, const int32_t* s_intro, int32_t np, int32_t p_len,
                                           const int32_t* p_nodes, const int32_t* p_offs, const int32_t* p_start,
                                           const int32_t* p_end, int32_t* EI, int32_t* NR, int32_t* NM, int32_t* NC,
                                           void* ws, size_t ws_bytes, void* stream) {
  if (n_depots < 1 || n_nodes <= n_depots || n_nodes > 65535) return fail(MDVRP_EINVAL, "bad node counts");
  if ((int64_t)ns * np > INT32_MAX) return fail(MDVRP_EINVAL, "too many route pairs");
  if (ns > 0 && !s_intro) return fail(MDVRP_EINVAL, "null intro flags");
  if ((int64_t)ns * np > 0 && (!EI || !NR || !NM || !NC)) return fail(MDVRP_EINVAL, "null output");
  hipStream_t s = S(stream);
  if (mdvrp_status e = check_routes_dev("offspring", n_depots, n_nodes, ns, s_len, s_nodes, s_offs, s_start, s_end,
                                        s_intro, false, s))
    return e;
  if (mdvrp_status e = check_routes_dev("parent", n_depots, n_nodes, np, p_len, p_nodes, p_offs, p_start, p_end,
                                        nullptr, true, s))
    return e;
  const size_t need = dcrex_ws_bytes(n_nodes, ns, np, p_len) + 256;
  if (!ws || ws_bytes < need) return fail(MDVRP_ENOSPC, "DCREX workspace needs %zu bytes", need);
  void* w = (void*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  int32_t* err = nullptr;
  launch_dcrex_counts(s, n_nodes, n_depots, ns, s_len, s_nodes, s_offs, s_start, s_end, s_intro, np, p_len, p_nodes,
                      p_offs, p_start, p_end, EI, NR, NM, NC, w, &err);
  HIP_TRY(hipGetLastError());
  int32_t h_err = 0;
  HIP_TRY(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h_err) return fail(MDVRP_ENOSPC, "a customer occurs in more than %d offspring routes", kOccMax);
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_dcrex_pick(int32_t ns, int32_t np, const int32_t* EI, const int32_t* NR,
                                         const int32_t* NM, const int32_t* NC, uint64_t seed, int32_t* out,
                                         void* stream) {
  if (ns < 0 || np < 0 || !out || ((int64_t)ns * np > 0 && (!EI || !NR || !NM || !NC)))
    return fail(MDVRP_EINVAL, "bad argument");
  if ((int64_t)ns * np > INT32_MAX) return fail(MDVRP_EINVAL, "too many route pairs");
  launch_dcrex_pick(S(stream), ns, np, EI, NR, NM, NC, seed, out);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_ucb_select(int32_t n_arms, const double* R, const double* N, int32_t* arm,
                                         void* stream) {
  if (n_arms < 1 || n_arms > 1024 || !R || !N || !arm) return fail(MDVRP_EINVAL, "bad argument");
  launch_ucb_select(S(stream), n_arms, R, N, arm);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_ucb_update(int32_t n_arms, double* R, double* N, const int32_t* arm,
                                         const double* reward, double gamma, void* stream) {
  if (n_arms < 1 || n_arms > 1024 || !R || !N || !arm || !reward || !(gamma > 0.0 && gamma <= 1.0))
    return fail(MDVRP_EINVAL, "bad argument");
  launch_ucb_update(S(stream), n_arms, R, N, arm, reward, gamma);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

static mdvrp_status batch_state(const mdvrp_batch* B, int64_t* out, void* stream) {
  const LaunchCtx L = B->ctx(stream);
  launch_state_export(L, B->d_state);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, B->d_state, sizeof(int64_t) * kStateWords * B->n_units, hipMemcpyDeviceToHost, L.stream));
  HIP_TRY(hipStreamSynchronize(L.stream));
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_batch_state(const mdvrp_batch* B, int64_t* out) {
  if (!B || !out) return fail(MDVRP_EINVAL, "null argument");
  HIP_TRY(hipDeviceSynchronize());
  return batch_state(B, out, nullptr);
}

// ============================================================================ hot path

// fmode: pair lists of the coming evaluations (0 full, 1 filtered); rescore = forget
// which routes the filtered lists reflect.
__global__ static void k_step_begin(const UnitDesc* units, int n_units, int fmode, int rescore) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_units) {
    UnitCtl* c = units[i].ctl;
    c->n_cand = 0;
    c->last_eval = 0;
    c->active = 1;
    c->fmode = fmode;
    if (rescore) c->scored_epoch = -1;
    c->t_start = (int64_t)wall_clock64();
    c->t_end = c->t_start;
  }
}

static void step_begin(const LaunchCtx& L, int fmode, int rescore) {
  hipLaunchKernelGGL(k_step_begin, dim3((L.n_units + 255) / 256), dim3(256), 0, L.stream, L.units, L.n_units, fmode,
                     rescore);
}

namespace {

// Host check of caller candidate lists (copied to the host): entries are customers of
// the unit's instance other than the anchor, or -1; no entry repeats within a list.
mdvrp_status check_cand_lists(const mdvrp_batch* B, const int32_t* cand, int32_t k, hipStream_t s) {
  int64_t total = 0;
  for (const UnitDesc& u : B->h_units) {
    if (k > u.theta) return fail(MDVRP_EINVAL, "candidate lists of %d entries exceed theta = %d", k, u.theta);
    total += (int64_t)u.nc * k;
  }
  std::vector<int32_t> h(std::max<int64_t>(total, 1));
  HIP_TRY(hipMemcpyAsync(h.data(), cand, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t at = 0;
  std::vector<int32_t> seen;
  for (int ui = 0; ui < B->n_units; ++ui) {
    const UnitDesc& u = B->h_units[ui];
    seen.assign(u.n, -1);
    for (int i = 0; i < u.nc; ++i, at += k)
      for (int j = 0; j < k; ++j) {
        const int v = h[at + j];
        if (v == -1) continue;
        if (v < u.nd || v >= u.n || v == u.nd + i)
          return fail(MDVRP_EINVAL, "unit %d customer %d: list entry %d is not another customer", ui, u.nd + i, v);
        if (seen[v] == i) return fail(MDVRP_EINVAL, "unit %d customer %d: entry %d repeats", ui, u.nd + i, v);
        seen[v] = i;
      }
  }
  return MDVRP_OK;
}

// Shared body of mdvrp_eval_neighbourhood and mdvrp_eval_dense.
mdvrp_status eval_impl(mdvrp_batch* B, uint32_t fam, const int32_t* cand, int32_t k, const mdvrp_moves* moves,
                       uint32_t flags, mdvrp_dense_rec* dense, int64_t dense_cap, unsigned long long* dense_count,
                       int64_t* n_evaluated, void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  if (fam & ~MDVRP_FAM_ALL) return fail(MDVRP_EINVAL, "unknown family bits");
  if (flags & ~MDVRP_EVAL_FILTERED) return fail(MDVRP_EINVAL, "unknown flags");
  if (cand && (flags & MDVRP_EVAL_FILTERED)) return fail(MDVRP_EINVAL, "caller lists and the filter's lists together");
  if (cand && k < 1) return fail(MDVRP_EINVAL, "candidate lists need k >= 1");
  if ((flags & MDVRP_EVAL_FILTERED) && B->kc == 0) return fail(MDVRP_ESTATE, "no filter attached");
  if (moves && (!moves->count || moves->cap < 0 || (moves->cap > 0 && (!moves->dF || !moves->dD || !moves->id ||
                !moves->kind || !moves->variant || !moves->changed || !moves->unit || !moves->a || !moves->b ||
                !moves->res))))
    return fail(MDVRP_EINVAL, "incomplete move list");
  static_assert(sizeof(mdvrp_dense_rec) == sizeof(DenseRec), "dense record layout");
  if (mdvrp_status e = need_loaded(B)) return e;
  hipStream_t s = S(stream);
  if (cand) {
    if (mdvrp_status e = check_cand_lists(B, cand, k, s)) return e;
    // point every unit at its slice of the caller's lists for this evaluation
    std::vector<UnitDesc> u = B->h_units;
    int64_t off = 0;
    for (UnitDesc& x : u) {
      x.fcand = const_cast<int32_t*>(cand) + off * k;
      x.kc = k;
      x.ftiles = (int32_t)(((int64_t)x.nc * k + kTileItems - 1) / kTileItems);
      off += x.nc;
    }
    HIP_TRY(hipMemcpyAsync(B->d_units, u.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (moves) HIP_TRY(hipMemsetAsync(moves->count, 0, sizeof(unsigned long long), s));
  LaunchCtx L = B->ctx(stream);
  const bool filt = cand || (flags & MDVRP_EVAL_FILTERED);
  L.compact = (flags & MDVRP_EVAL_FILTERED) ? 1 : 0;
  step_begin(L, filt ? 1 : 0, 0);
  DenseOut D{};
  D.rec = (DenseRec*)dense;
  D.count = dense_count;
  D.cap = dense_cap;
  if (moves) {
    D.ml.dF = moves->dF; D.ml.dD = moves->dD; D.ml.id = moves->id; D.ml.kind = moves->kind;
    D.ml.variant = moves->variant; D.ml.changed = moves->changed; D.ml.unit = moves->unit;
    D.ml.a = moves->a; D.ml.b = moves->b; D.ml.res = moves->res; D.ml.cap = moves->cap; D.ml.count = moves->count;
  }
  const bool sink = dense || moves;
  const uint32_t cls = eval_classes(L, fam);
  for (int c = 0; c < 3; ++c)
    if (cls >> c & 1)
      timed(B, L.stream, c, [&] { launch_eval_class(L, fam, c, sink ? &D : nullptr, sink ? 0 : B->shape_for(fam)); });
  HIP_TRY(hipGetLastError());
  if (n_evaluated) launch_evaluated_export(L, n_evaluated);
  B->planned = false;
  B->eval_fam = fam;
  if (cand) {
    HIP_TRY(hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (moves) {
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, moves->count, sizeof n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((int64_t)n > moves->cap)
      return fail(MDVRP_ENOSPC, "the move list needs %llu rows (capacity %lld)", n, (long long)moves->cap);
  }
  return MDVRP_OK;
}

}  // namespace

extern "C" mdvrp_status mdvrp_eval_neighbourhood(mdvrp_batch* B, uint32_t fam, const int32_t* cand, int32_t k,
                                                 mdvrp_moves* moves, uint32_t flags, int64_t* n_evaluated,
                                                 void* stream) {
  return eval_impl(B, fam, cand, k, moves, flags, nullptr, 0, nullptr, n_evaluated, stream);
}

extern "C" mdvrp_status mdvrp_eval_dense(mdvrp_batch* B, uint32_t fam, uint32_t flags, mdvrp_dense_rec* dense,
                                         int64_t dense_cap, unsigned long long* dense_count, void* stream) {
  if (!dense || !dense_count || dense_cap < 0) return fail(MDVRP_EINVAL, "dense output needs a buffer and a counter");
  return eval_impl(B, fam, nullptr, 0, nullptr, flags, dense, dense_cap, dense_count, nullptr, stream);
}

extern "C" mdvrp_status mdvrp_eval_footprint(mdvrp_batch* B, uint32_t fam, uint32_t* bitmap, int64_t words,
                                             void* stream) {
  if (!B || !bitmap) return fail(MDVRP_EINVAL, "null argument");
  if (fam & ~MDVRP_FAM_ALL) return fail(MDVRP_EINVAL, "unknown family bits");
  std::vector<int64_t> base(B->inst.size() + 1, 0);
  for (size_t k = 0; k < B->inst.size(); ++k) {
    const int64_t n = B->inst[k]->N;
    base[k + 1] = base[k] + (n * n + 31) / 32;
  }
  if (words < base.back()) return fail(MDVRP_ENOSPC, "footprint bitmap needs %lld words", (long long)base.back());
  if (mdvrp_status e = need_loaded(B)) return e;
  B->state_changed();
  hipStream_t s = S(stream);
  std::vector<UnitDesc> u = B->h_units;
  for (int k = 0; k < B->n_units; ++k) u[k].foot = bitmap + base[B->unit_inst[k]];
  HIP_TRY(hipMemcpyAsync(B->d_units, u.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
  const LaunchCtx L = B->ctx(stream);
  step_begin(L, 0, 0);
  const uint32_t cls = eval_classes(L, fam);
  for (int c = 0; c < 3; ++c)
    if (cls >> c & 1) launch_eval_footprint(L, fam, c);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
  step_begin(L, 0, 0);
  HIP_TRY(hipStreamSynchronize(s));
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_select_multimove(mdvrp_batch* B, uint32_t fam, int32_t leader_only, uint64_t* sel_ids,
                                               int64_t* sel_dF, int32_t* sel_count, int32_t sel_cap, void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  if (sel_ids && (!sel_dF || !sel_count || sel_cap < 1)) return fail(MDVRP_EINVAL, "selection output incomplete");
  if (mdvrp_status e = need_loaded(B)) return e;
  const LaunchCtx L = B->ctx(stream);
  if (fam == 0 || fam != B->eval_fam)
    return fail(MDVRP_ESTATE, "select: the latest evaluation of the current solutions was not of these families");
  B->eval_fam = 0;
  B->planned = true;
  timed(B, L.stream, 3, [&] { launch_select(L, fam, leader_only ? 1 : 0); });
  if (sel_ids) launch_sel_export(L, sel_ids, sel_dF, sel_count, sel_cap);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_apply_moves(mdvrp_batch* B, void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  if (!B->planned) return fail(MDVRP_ESTATE, "apply: no selection to apply");
  const LaunchCtx L = B->ctx(stream);
  B->state_changed();
  timed(B, L.stream, 4, [&] { launch_rebuild(L); });
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

static mdvrp_status check_unit_errors(mdvrp_batch* B, std::vector<int64_t>& st, void* stream) {
  st.resize((size_t)B->n_units * kStateWords);
  mdvrp_status s = batch_state(B, st.data(), stream);
  if (s) return s;
  for (int k = 0; k < B->n_units; ++k) {
    const int64_t e = st[(size_t)k * kStateWords + 5];
    if (e & 4) return fail(MDVRP_ERANGE, "unit %d: a route exceeded the int32-safe length", k);
    if (e & 3) return fail(MDVRP_ENOSPC, "unit %d: internal capacity exceeded (bits %lld)", k, (long long)e);
    if (e) return fail(MDVRP_ESTATE, "unit %d: internal invariant failed (bits %lld)", k, (long long)e);
  }
  return MDVRP_OK;
}

namespace {

// Launch sequence of one pass of the local search (Algorithm 2): the families in
// the pass's order, each evaluated, selected and applied; optional re-ranking of
// the filtered lists. With time = false nothing is timed (graph capture).
void launch_pass(mdvrp_batch* B, const LaunchCtx& L, const mdvrp_ls_options* o, const int32_t* fam, int nf,
                 int64_t pass, bool time) {
  const uint32_t pair_fams = MDVRP_FAM_RELOCATE | MDVRP_FAM_SWAP | MDVRP_FAM_2OPT_STAR | MDVRP_FAM_2OPT;
  const bool rescoring = o->filter == MDVRP_FILTER_MLP;
  auto run = [&](int cls, auto&& f) {
    if (time) timed(B, L.stream, cls, f);
    else f();
  };
  launch_pass_begin(L);
  bool ranked_this_pass = false;
  for (int k = 0; k < nf; ++k) {
    const uint32_t mask = o->mode == MDVRP_LS_PASSES ? (1u << fam[k]) : MDVRP_FAM_ALL;
    const uint32_t cls = eval_classes(L, mask);
    // re-rank the lists of filtered units whose features changed since the last ranking:
    // before every pair-family step, or before the first one of every rescore-th pass
    const bool pair_step = (mask & pair_fams) && (cls & 1u);
    const bool rank_pass = o->rescore == MDVRP_RESCORE_STEP || pass % o->rescore == 0;
    const bool score = rescoring && pair_step && rank_pass && !(o->rescore > 0 && ranked_this_pass);
    if (pair_step) ranked_this_pass = true;
    if (score)
      run(MDVRP_PROF_FILTER_SCORE,
          [&] { launch_rank(L, B->d_cust_off, B->n_cust, o->mlp->d, B->stale, 0); });
    for (int c = 0; c < 3; ++c)
      if (cls >> c & 1) run(c, [&] { launch_eval_class(L, mask, c, nullptr, B->shape_for(mask)); });
    run(3, [&] { launch_select(L, mask, o->leader_only ? 1 : 0, score ? 1 : 0, /*apply=*/true); });
  }
  launch_pass_end(L);
}

}  // namespace

extern "C" mdvrp_status mdvrp_local_search_to_optimum(mdvrp_batch* B, const mdvrp_ls_options* o,
                                                      mdvrp_ls_stats* stats, void* stream) {
  if (!B || !o) return fail(MDVRP_EINVAL, "null argument");
  if (o->mode != MDVRP_LS_PASSES && o->mode != MDVRP_LS_UNION) return fail(MDVRP_EINVAL, "unknown mode");
  if (o->max_passes < 0) return fail(MDVRP_EINVAL, "max_passes must be >= 0");
  if (o->filter < MDVRP_FILTER_NONE || o->filter > MDVRP_FILTER_MLP) return fail(MDVRP_EINVAL, "unknown filter");
  if (o->filter != MDVRP_FILTER_NONE && B->kc == 0) return fail(MDVRP_ESTATE, "no filter attached to the batch");
  if (o->filter == MDVRP_FILTER_MLP && !o->mlp) return fail(MDVRP_EINVAL, "the MLP filter needs a network");
  if (o->rescore < 0) return fail(MDVRP_EINVAL, "rescore must be >= 0");
  if (o->graph != 0 && o->graph != 1) return fail(MDVRP_EINVAL, "graph must be 0 or 1");
  if (o->penalty_adapt != 0 && o->penalty_adapt != 1) return fail(MDVRP_EINVAL, "penalty_adapt must be 0 or 1");
  if (o->penalty_adapt && o->max_passes == 0)
    return fail(MDVRP_EINVAL, "penalty_adapt needs a search depth (max_passes > 0): with moving weights a search "
                              "can revisit solutions forever");
  if (o->penalty_adapt)
    for (int k = 0; k < 4; ++k)
      if (o->w_min[k] < 0 || o->w_min[k] > o->w_max[k] || o->w_max[k] > (1 << 30))
        return fail(MDVRP_EINVAL, "weight %d: bounds [%d, %d] outside 0 <= w_min <= w_max <= 2^30", k, o->w_min[k],
                    o->w_max[k]);
  if (mdvrp_status e = need_loaded(B)) return e;
  B->state_changed();
  const int poll = std::max(1, o->poll_every);
  // A pass captured as a graph needs a capturable stream: the null stream is
  // replaced by the batch's own stream, ordered after and before the caller's work.
  hipStream_t st = S(stream);
  const bool use_own = o->graph && st == nullptr;
  if (use_own) {
    if (!B->own) {
      HIP_TRY(hipStreamCreateWithFlags(&B->own, hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(B->ev_in, st));
    HIP_TRY(hipStreamWaitEvent(B->own, B->ev_in, 0));
    st = B->own;
  }
  LaunchCtx L = B->ctx(st);
  L.compact = o->filter != MDVRP_FILTER_NONE;
  B->search_grids(L);
  if (o->penalty_adapt) {
    // every unit starts from its instance's weights; the fused steps adapt them on the device
    if (weights_to_instance(B))
      HIP_TRY(hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, st));
    L.adapt_units = B->d_units;
    for (int k = 0; k < 4; ++k) {
      L.adapt.lo[k] = o->w_min[k];
      L.adapt.hi[k] = o->w_max[k];
    }
  }
  step_begin(L, o->filter != MDVRP_FILTER_NONE ? 1 : 0, o->filter == MDVRP_FILTER_MLP ? 1 : 0);
  if (!B->h_poll) {
    HIP_TRY(hipHostMalloc((void**)&B->h_poll, 2 * sizeof(int32_t), hipHostMallocDefault));
    for (hipEvent_t& e : B->ev_poll) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // Pipelined convergence check: at the end of poll interval c the active-unit count is
  // copied to host slot c % 2; the host then waits for interval c - 1's copy, which the
  // GPU finished before starting interval c, so the queue never drains. Passes that run
  // after the last unit converged are no-ops (every kernel skips inactive units).
  int64_t chunk = 0;
  for (int64_t p = 0; o->max_passes == 0 || p < o->max_passes; ++p) {
    int32_t fam[6];
    const int nf = o->mode == MDVRP_LS_PASSES ? mdvrp_family_order(B->has_tw, o->seed, p, fam) : 1;
    if (!o->graph) {
      launch_pass(B, L, o, fam, nf, p, true);
    } else {
      const int64_t rank_phase = o->rescore > 0 ? (p % o->rescore == 0) : 0;
      std::vector<int64_t> key = {o->mode, o->leader_only, o->filter, o->rescore, rank_phase, (int64_t)(intptr_t)o->mlp,
                                  o->penalty_adapt, nf};
      if (o->penalty_adapt)
        for (int k = 0; k < 4; ++k) {
          key.push_back(o->w_min[k]);
          key.push_back(o->w_max[k]);
        }
      for (int k = 0; k < nf; ++k) key.push_back(fam[k]);
      auto it = B->graphs.find(key);
      if (it == B->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        launch_pass(B, L, o, fam, nf, p, false);
        HIP_TRY(hipStreamEndCapture(st, &g));
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(MDVRP_EDEVICE, "graph instantiation: %s", hipGetErrorString(e));
        it = B->graphs.emplace(key, ex).first;
      }
      HIP_TRY(hipGraphLaunch(it->second, st));
    }
    HIP_TRY(hipGetLastError());
    if ((p + 1) % poll == 0) {
      const int slot = (int)(chunk & 1);
      HIP_TRY(hipMemcpyAsync(&B->h_poll[slot], B->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipEventRecord(B->ev_poll[slot], st));
      if (chunk > 0) {
        HIP_TRY(hipEventSynchronize(B->ev_poll[slot ^ 1]));
        if (B->h_poll[slot ^ 1] == 0) break;
      }
      ++chunk;
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  launch_cost(L, nullptr, nullptr);  // F under the weights the search ended with
  std::vector<int64_t> stv;
  mdvrp_status s = check_unit_errors(B, stv, st);
  if (o->penalty_adapt && s != MDVRP_EDEVICE)
    for (int k = 0; k < B->n_units; ++k) {  // keep the host copy of the descriptors in step
      const int64_t* x = &stv[(size_t)k * kStateWords];
      UnitDesc& u = B->h_units[k];
      u.w_tw = (int32_t)x[12];
      u.w_load = (int32_t)x[13];
      u.w_dur = (int32_t)x[14];
      u.w_depot = x[15];
    }
  if (use_own) {
    HIP_TRY(hipEventRecord(B->ev_out, st));
    HIP_TRY(hipStreamWaitEvent(S(stream), B->ev_out, 0));
  }
  if (stats) {
    for (int k = 0; k < B->n_units; ++k) {
      const int64_t* x = &stv[(size_t)k * kStateWords];
      stats[k].F = x[0];
      stats[k].evaluated = x[1];
      stats[k].passes = x[2];
      stats[k].steps = x[3];
      stats[k].moves_applied = x[4];
      stats[k].fallback_passes = x[8];
      stats[k].device_ms = B->clock_khz > 0 ? (double)(x[11] - x[10]) / B->clock_khz : -1.0;
      stats[k].err = (int32_t)x[5];
      stats[k].converged = x[6] ? 0 : 1;
      for (int w = 0; w < 4; ++w) stats[k].w_final[w] = x[12 + w];
    }
  }
  return s;
}

// ============================================================================ autotuner

__global__ static void k_restore_counts(const UnitDesc* units, int n_units, const int64_t* saved) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_units) {
    units[i].ctl->evaluated = saved[(int64_t)i * kStateWords + 1];
    units[i].ctl->last_eval = 0;
    units[i].ctl->n_cand = 0;
  }
}

extern "C" mdvrp_status mdvrp_autotune(mdvrp_batch* B, uint32_t fam_mask, int32_t reps, int32_t* shapes_out,
                                       void* stream) {
  if (!B || reps < 1) return fail(MDVRP_EINVAL, "bad argument");
  if (fam_mask & ~MDVRP_FAM_ALL) return fail(MDVRP_EINVAL, "unknown family bits");
  if (mdvrp_status e = need_loaded(B)) return e;
  B->state_changed();
  const LaunchCtx L = B->ctx(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  launch_state_export(L, B->d_state);  // evaluation counters, restored below
  mdvrp_status st = MDVRP_OK;
  for (int f = 0; f < 6 && st == MDVRP_OK; ++f) {
    const uint32_t mask = 1u << f;
    const uint32_t cls = eval_classes(L, mask);
    if (!(fam_mask & mask) || !cls) continue;
    const int c = cls & 1u ? 0 : (cls & 2u ? 1 : 2);
    float best_ms = 0;
    int best = 0;
    for (int shape = 0; shape < kNumTileShapes; ++shape) {
      step_begin(L, 0, 0);
      launch_eval_class(L, mask, c, nullptr, shape);  // warm-up
      step_begin(L, 0, 0);
      (void)hipEventRecord(e0, L.stream);
      for (int r = 0; r < reps; ++r) {
        launch_eval_class(L, mask, c, nullptr, shape);
        step_begin(L, 0, 0);
      }
      (void)hipEventRecord(e1, L.stream);
      hipError_t he = hipEventSynchronize(e1);
      float ms = 0;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) { st = fail(MDVRP_EDEVICE, "autotune: %s", hipGetErrorString(he)); break; }
      if (shape == 0 || ms < best_ms) { best_ms = ms; best = shape; }
    }
    B->shape[f] = best;
  }
  hipLaunchKernelGGL(k_restore_counts, dim3((B->n_units + 255) / 256), dim3(256), 0, L.stream, L.units, B->n_units,
                     (const int64_t*)B->d_state);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->drop_graphs();  // captured passes hold the previous shapes
  if (st) return st;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(L.stream));
  if (shapes_out)
    for (int f = 0; f < 6; ++f) shapes_out[f] = tile_shape_threads(B->shape[f]);
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_set_tile_shapes(mdvrp_batch* B, const int32_t* threads) {
  if (!B || !threads) return fail(MDVRP_EINVAL, "null argument");
  int sh[6];
  for (int f = 0; f < 6; ++f) {
    sh[f] = -1;
    for (int k = 0; k < kNumTileShapes; ++k)
      if (tile_shape_threads(k) == threads[f]) sh[f] = k;
    if (sh[f] < 0) return fail(MDVRP_EINVAL, "family %d: no tile shape with %d threads", f, threads[f]);
  }
  for (int f = 0; f < 6; ++f) B->shape[f] = sh[f];
  B->drop_graphs();
  return MDVRP_OK;
}

// ============================================================================ learned move filter

namespace {

void carve_mlp(Carve& cv, MlpDev* M) {
  const int np = mlp_param_count();
  MlpDev m{};
  m.P = cv.take<float>(np);
  m.m = cv.take<float>(np);
  m.v = cv.take<float>(np);
  m.w1f = cv.take<char>(16 * 64 * 16);
  m.w2f = cv.take<char>(16 * 8 * 64 * 16);
  m.w2b = cv.take<char>(16 * 8 * 64 * 16);
  m.w3b = cv.take<float>(256);
  m.scratch = cv.take<float>(2 + kBceBlocks);
  if (M) *M = m;
}

struct ActBufs {
  uint16_t *h1, *h2, *G2, *G1;
  float* dz;
  float* part;  // partial sums of the backward pass
};

// Activation workspace of n samples: h1, h2 (rows padded for the forward tiles), the
// two backward gradients, dlogits, and the backward pass's partial sums.
void carve_act(Carve& cv, int n, ActBufs* A) {
  const int pad = mlp_row_pad();
  const size_t rows = ((size_t)std::max(n, 1) + pad - 1) / pad * pad;
  ActBufs a{};
  a.h1 = cv.take<uint16_t>(rows * 256);
  a.h2 = cv.take<uint16_t>(rows * 256);
  a.G2 = cv.take<uint16_t>(rows * 256);
  a.G1 = cv.take<uint16_t>(rows * 256);
  a.dz = cv.take<float>(rows);
  a.part = cv.take<float>(mlp_grad_part_floats(n));
  if (A) *A = a;
}

mdvrp_status check_act(int32_t n, void* act_ws, size_t act_bytes, ActBufs* A) {
  Carve need(nullptr);
  carve_act(need, n, nullptr);
  if (!act_ws || act_bytes < need.off + 256)
    return fail(MDVRP_ENOSPC, "activation workspace needs %zu bytes", need.off + 256);
  Carve cv(act_ws);
  carve_act(cv, n, A);
  return MDVRP_OK;
}

}  // namespace

extern "C" mdvrp_status mdvrp_mlp_workspace_query(size_t* bytes) {
  if (!bytes) return fail(MDVRP_EINVAL, "null bytes");
  Carve cv(nullptr);
  carve_mlp(cv, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_create(void* ws, size_t ws_bytes, const float* params_init, void* stream,
                                         mdvrp_mlp** out) {
  if (!out) return fail(MDVRP_EINVAL, "null out");
  size_t need = 0;
  mdvrp_mlp_workspace_query(&need);
  if (!ws || ws_bytes < need) return fail(MDVRP_ENOSPC, "MLP workspace needs %zu bytes", need);
  mdvrp_mlp* M = new mdvrp_mlp();
  Carve cv(ws);
  carve_mlp(cv, &M->d);
  const int np = mlp_param_count();
  hipStream_t s = S(stream);
  hipError_t he = hipSuccess;
  if (params_init)
    he = hipMemcpyAsync(M->d.P, params_init, sizeof(float) * np, hipMemcpyDeviceToDevice, s);
  else
    launch_mlp_zero(s, M->d.P, np);
  launch_mlp_zero(s, M->d.m, np);
  launch_mlp_zero(s, M->d.v, np);
  launch_mlp_pack(s, M->d);
  if (he == hipSuccess) he = hipGetLastError();
  if (he != hipSuccess) {
    delete M;
    return fail(MDVRP_EDEVICE, "MLP create: %s", hipGetErrorString(he));
  }
  *out = M;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_params(mdvrp_mlp* M, float** params) {
  if (!M || !params) return fail(MDVRP_EINVAL, "null argument");
  *params = M->d.P;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_sync(mdvrp_mlp* M, int32_t reset_adam, void* stream) {
  if (!M) return fail(MDVRP_EINVAL, "null network");
  const int np = mlp_param_count();
  if (reset_adam) {
    launch_mlp_zero(S(stream), M->d.m, np);
    launch_mlp_zero(S(stream), M->d.v, np);
  }
  launch_mlp_pack(S(stream), M->d);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" void mdvrp_mlp_destroy(mdvrp_mlp* M) { delete M; }

extern "C" mdvrp_status mdvrp_mlp_act_bytes(int32_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(MDVRP_EINVAL, "bad argument");
  Carve cv(nullptr);
  carve_act(cv, n, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_forward(const mdvrp_mlp* M, const uint16_t* x, int32_t n, float* logits,
                                          void* act_ws, size_t act_bytes, void* stream) {
  if (!M || n < 0 || (n > 0 && (!x || !logits))) return fail(MDVRP_EINVAL, "bad argument");
  ActBufs A{};
  if (act_ws) {
    mdvrp_status st = check_act(n, act_ws, act_bytes, &A);
    if (st) return st;
  }
  launch_mlp_forward(S(stream), M->d, x, n, logits, act_ws ? A.h1 : nullptr, act_ws ? A.h2 : nullptr);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_backward(const mdvrp_mlp* M, const uint16_t* x, const float* dlogits, int32_t n,
                                           float* grads, void* act_ws, size_t act_bytes, void* stream) {
  if (!M || !grads || n < 0 || (n > 0 && (!x || !dlogits))) return fail(MDVRP_EINVAL, "bad argument");
  ActBufs A{};
  mdvrp_status st = check_act(n, act_ws, act_bytes, &A);
  if (st) return st;
  launch_mlp_backward(S(stream), M->d, x, n, dlogits, A.h1, A.h2, grads, A.G2, A.G1, A.part);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_bce(mdvrp_mlp* M, const float* logits, const float* labels, const float* weights,
                                      int32_t n, float* dlogits, float* loss, void* stream) {
  if (!M || n < 0 || (n > 0 && (!logits || !labels || !dlogits))) return fail(MDVRP_EINVAL, "bad argument");
  launch_bce(S(stream), logits, labels, weights, n, M->d.scratch, bce_blocks(n, kBceBlocks), dlogits, loss);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_adam_step(mdvrp_mlp* M, const float* grads, float lr, int32_t step, void* stream) {
  if (!M || !grads || step < 1 || !(lr >= 0.f)) return fail(MDVRP_EINVAL, "bad argument");
  launch_adam(S(stream), M->d, grads, lr, step);
  launch_mlp_pack(S(stream), M->d);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_mlp_train_step(mdvrp_mlp* M, const uint16_t* x, const float* labels,
                                             const float* weights, int32_t n, float lr, int32_t step, float* grads,
                                             float* logits, float* loss, void* act_ws, size_t act_bytes,
                                             void* stream) {
  if (!M || !x || !labels || !grads || !logits || n < 1 || step < 1 || !(lr >= 0.f))
    return fail(MDVRP_EINVAL, "bad argument");
  ActBufs A{};
  mdvrp_status st = check_act(n, act_ws, act_bytes, &A);
  if (st) return st;
  hipStream_t s = S(stream);
  launch_mlp_forward(s, M->d, x, n, logits, A.h1, A.h2);
  launch_bce(s, logits, labels, weights, n, M->d.scratch, bce_blocks(n, kBceBlocks), A.dz, loss);
  launch_mlp_backward(s, M->d, x, n, A.dz, A.h1, A.h2, grads, A.G2, A.G1, A.part);
  launch_adam(s, M->d, grads, lr, step);
  launch_mlp_pack(s, M->d);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

// ---------------------------------------------------------------------------- allocation-free training step
//
// mdvrp_mlp_train_step_static keeps the activations, gradients of the hidden layers
// and the backward pass's partial sums -- the act_ws of mdvrp_mlp_train_step -- in
// this file-scope device array. Each GPU the library runs on holds its own copy until
// the process ends. On the host the array's name is only a stand-in symbol: every
// host use goes through the device address hipGetSymbolAddress returns for the
// current device, looked up once per device on the entry point's first call there.
constexpr int kStaticTrainMaxN = MDVRP_TRAIN_STATIC_MAX_N;
constexpr size_t kStaticTrainBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticTrainBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

mdvrp_status static_scratch(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MDVRP_EDEVICE, "device %d beyond the static scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MDVRP_EDEVICE, "no device address for the static scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MDVRP_OK;
}

}  // namespace

extern "C" mdvrp_status mdvrp_mlp_train_step_static(mdvrp_mlp* M, const uint16_t* x, const float* labels,
                                                    const float* weights, int32_t n, float lr, int32_t step,
                                                    float* grads, float* logits, float* loss, void* stream) {
  if (!M || !x || !labels || !grads || !logits || n < 1 || step < 1 || !(lr >= 0.f))
    return fail(MDVRP_EINVAL, "bad argument");
  if (n > kStaticTrainMaxN)
    return fail(MDVRP_EINVAL, "mdvrp_mlp_train_step_static takes at most %d samples per call (got %d)",
                kStaticTrainMaxN, n);
  Carve need(nullptr);
  carve_act(need, n, nullptr);
  if (need.off + 256 > kStaticTrainBytes)
    return fail(MDVRP_ESTATE, "static scratch of %zu bytes is below the %zu bytes of %d samples", kStaticTrainBytes,
                need.off + 256, n);
  void* ws = nullptr;
  mdvrp_status st = static_scratch(&ws);
  if (st) return st;
  ActBufs A{};
  Carve cv(ws);
  carve_act(cv, n, &A);
  hipStream_t s = S(stream);
  launch_mlp_forward(s, M->d, x, n, logits, A.h1, A.h2);
  launch_bce(s, logits, labels, weights, n, M->d.scratch, bce_blocks(n, kBceBlocks), A.dz, loss);
  launch_mlp_backward(s, M->d, x, n, A.dz, A.h1, A.h2, grads, A.G2, A.G1, A.part);
  launch_adam(s, M->d, grads, lr, step);
  launch_mlp_pack(s, M->d);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

// ---------------------------------------------------------------------------- filter on a batch

namespace {

mdvrp_status check_filter_k(const mdvrp_batch* B, int32_t k) {
  if (k < 1) return fail(MDVRP_EINVAL, "list length must be >= 1");
  if (B->n_anchors >= INT32_MAX) return fail(MDVRP_ERANGE, "more than 2^31 - 1 anchors in one batch");
  for (const mdvrp_instance* I : B->inst)
    if (k > I->d.theta) return fail(MDVRP_EINVAL, "list length %d exceeds theta %d", k, I->d.theta);
  return MDVRP_OK;
}

void carve_filter(Carve& cv, const mdvrp_batch* B, int32_t k, std::vector<int32_t*>* lists, int32_t** cust_off,
                  FilterQueue* stale, int32_t** tile_off_f = nullptr) {
  int32_t* co = cv.take<int32_t>(B->n_units + 1);
  if (cust_off) *cust_off = co;
  int32_t* tf = cv.take<int32_t>(B->n_units + 1);
  if (tile_off_f) *tile_off_f = tf;
  FilterQueue q{};
  q.lcache = cv.take<float>(B->n_anchors);
  q.queue = cv.take<int32_t>(B->n_anchors);
  q.count = cv.take<int32_t>(1);
  q.cmark = cv.take<uint8_t>(B->n_cust);
  q.anchor_off = cv.take<int64_t>(B->n_units + 1);
  q.n_anchors = B->n_anchors;
  q.max_unit_anchors = 0;
  for (const UnitDesc& U : B->h_units) q.max_unit_anchors = std::max<int64_t>(q.max_unit_anchors, (int64_t)U.nc * U.theta);
  if (stale) *stale = q;
  for (int u = 0; u < B->n_units; ++u) {
    int32_t* p = cv.take<int32_t>((size_t)B->inst[B->unit_inst[u]]->d.n_customers * k);
    if (lists) lists->push_back(p);
  }
}

}  // namespace

extern "C" mdvrp_status mdvrp_filter_workspace_query(const mdvrp_batch* B, int32_t k, size_t* bytes) {
  if (!B || !bytes) return fail(MDVRP_EINVAL, "null argument");
  mdvrp_status st = check_filter_k(B, k);
  if (st) return st;
  Carve cv(nullptr);
  carve_filter(cv, B, k, nullptr, nullptr, nullptr);
  *bytes = cv.off + 256;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_attach(mdvrp_batch* B, int32_t k, void* ws, size_t ws_bytes, void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  mdvrp_status st = check_filter_k(B, k);
  if (st) return st;
  size_t need = 0;
  mdvrp_filter_workspace_query(B, k, &need);
  if (!ws || ws_bytes < need) return fail(MDVRP_ENOSPC, "filter workspace needs %zu bytes", need);
  Carve cv(ws);
  std::vector<int32_t*> lists;
  int32_t* co = nullptr;
  int32_t* tf = nullptr;
  FilterQueue fq{};
  carve_filter(cv, B, k, &lists, &co, &fq, &tf);
  std::vector<int32_t> h_co(B->n_units + 1, 0), h_tf(B->n_units + 1, 0);
  std::vector<int64_t> h_ao(B->n_units + 1, 0);
  for (int u = 0; u < B->n_units; ++u) h_ao[u + 1] = h_ao[u] + (int64_t)B->h_units[u].nc * B->h_units[u].theta;
  for (int u = 0; u < B->n_units; ++u) {
    UnitDesc& U = B->h_units[u];
    U.fcand = lists[u];
    U.kc = k;
    U.ftiles = (int32_t)(((int64_t)U.nc * k + kTileItems - 1) / kTileItems);
    h_co[u + 1] = h_co[u] + U.nc;
    h_tf[u + 1] = h_tf[u] + U.ftiles;
  }
  hipStream_t s = S(stream);
  HIP_TRY(hipMemcpyAsync(co, h_co.data(), sizeof(int32_t) * (B->n_units + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(tf, h_tf.data(), sizeof(int32_t) * (B->n_units + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync((void*)fq.anchor_off, h_ao.data(), sizeof(int64_t) * (B->n_units + 1), hipMemcpyHostToDevice,
                         s));
  HIP_TRY(hipMemsetAsync(fq.cmark, 0, B->n_cust, s));
  HIP_TRY(hipMemcpyAsync(B->d_units, B->h_units.data(), sizeof(UnitDesc) * B->n_units, hipMemcpyHostToDevice, s));
  B->drop_graphs();  // captured passes refer to the previous filter state
  B->kc = k;
  B->d_cust_off = co;
  B->d_tile_off_f = tf;
  B->h_tile_off_f = h_tf;
  B->stale = fq;
  // start from the heuristic lists so that a filtered evaluation is always defined
  launch_eta_lists(B->ctx(stream), co, B->n_cust);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_anchor_count(const mdvrp_batch* B, int64_t* n) {
  if (!B || !n) return fail(MDVRP_EINVAL, "null argument");
  *n = B->n_anchors;
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_features(mdvrp_batch* B, uint16_t* feats, void* stream) {
  if (!B || !feats) return fail(MDVRP_EINVAL, "null argument");
  if (mdvrp_status e = need_loaded(B)) return e;
  launch_features(B->ctx(stream), feats);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_labels(mdvrp_batch* B, uint32_t fam, uint8_t* labels, void* stream) {
  if (!B || !labels) return fail(MDVRP_EINVAL, "null argument");
  if (fam & ~MDVRP_FAM_ALL) return fail(MDVRP_EINVAL, "unknown family bits");
  if (mdvrp_status e = need_loaded(B)) return e;
  B->state_changed();
  const LaunchCtx L = B->ctx(stream);
  step_begin(L, 0, 0);
  DenseOut D;
  D.label = labels;
  if (eval_classes(L, fam) & 1u) launch_eval_class(L, fam, 0, &D);
  step_begin(L, 0, 0);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_score_topk(mdvrp_batch* B, const mdvrp_mlp* M, float* logits, void* stream) {
  if (!B || !M) return fail(MDVRP_EINVAL, "null argument");
  if (B->kc == 0) return fail(MDVRP_ESTATE, "no filter attached");
  if (mdvrp_status e = need_loaded(B)) return e;
  const LaunchCtx L = B->ctx(stream);
  timed(B, L.stream, MDVRP_PROF_FILTER_SCORE, [&] { launch_rank(L, B->d_cust_off, B->n_cust, M->d, B->stale, 1); });
  if (logits)
    HIP_TRY(hipMemcpyAsync(logits, B->stale.lcache, sizeof(float) * B->n_anchors, hipMemcpyDeviceToDevice, L.stream));
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_eta_lists(mdvrp_batch* B, void* stream) {
  if (!B) return fail(MDVRP_EINVAL, "null batch");
  if (B->kc == 0) return fail(MDVRP_ESTATE, "no filter attached");
  launch_eta_lists(B->ctx(stream), B->d_cust_off, B->n_cust);
  HIP_TRY(hipGetLastError());
  return MDVRP_OK;
}

extern "C" mdvrp_status mdvrp_filter_export(const mdvrp_batch* B, int32_t* cand, void* stream) {
  if (!B || !cand) return fail(MDVRP_EINVAL, "null argument");
  if (B->kc == 0) return fail(MDVRP_ESTATE, "no filter attached");
  size_t at = 0;
  for (int u = 0; u < B->n_units; ++u) {
    const size_t n = (size_t)B->h_units[u].nc * B->kc;
    HIP_TRY(hipMemcpyAsync(cand + at, B->h_units[u].fcand, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, S(stream)));
    at += n;
  }
  return MDVRP_OK;
}
