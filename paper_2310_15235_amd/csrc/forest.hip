// Batches of independent scenes (a forest) for the mean intensity path.
//
// Each scene is an ordinary radiation tree built in its slice of one
// workspace; a device table holds the scenes' DevTrees with the offsets of
// their blocks in the concatenated element, band and node arrays.  The
// per-bucket kernels of the forward and of the adjoint then run as one
// persistent launch per band count over the (scene, bucket) work items of
// every scene with that many bands; the number of active buckets and all
// per-bucket offsets stay on the device.
//
// A plan, made once per forest, fixes every size a call can need: the bucket
// setup (p-p radii and sets) and the walks do not depend on the active set
// (the p-p radius is set by every member of a bucket), so the all-active
// setup bounds the p-p lists, p-p columns and pair depths of any active set,
// and its longest cut list and traversal depth are those of every call.
// With the plan, compute_J_batched and compute_J_backward_batched enqueue
// kernels only: no synchronisation, allocation or memset, so a HIP graph can
// capture them.

#include <algorithm>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "path_device.hpp"
#include "path_host.hpp"

struct trevr_forest {
  uint64_t magic;
  int32_t S;
  std::vector<trevr_params> params;
  std::vector<int64_t> off;            // element offsets [S + 1]
  std::vector<trevr_tree*> trees;
  hipStream_t stream;
  void* ws;
  size_t ws_bytes;
  trevr::DevTree* dtab;                // device table [S]
  uint32_t* ferr;                      // device error bits of batched calls
  uint32_t* host;                      // pinned readback buffer
  int64_t n_total, jn_total, nodes_total, nodesB_total, alpha_total, leaves_total;
  int64_t max_nodes, max_n;
  int32_t bands_total;
  bool any_bg;
  std::vector<int64_t> level_work;     // widest scene's nodes x classes per depth
  int64_t class_leaves[trevr::kMaxBands];
  bool any_complex;                    // a scene uses the complex source model
  // plan
  bool planned;
  bool stack_large;
  uint32_t cut_cap;
  uint64_t tot[trevr::TOT_N];
  size_t scratch_run;
  size_t job_log_bytes;                // p-p job log asked for (trevr_forest_job_log)
  // the scratch holding the last batched forward state of this forest
  const void* fwd_scratch;
  uint64_t fwd_epoch;
  trevr::LaunchCfg cfg;                // launch options (trevr_forest_autotune)
  int32_t cfg_index;
  trevr::Prof prof;                    // kernel timing (trevr_forest_profile_enable)
};

namespace trevr {
namespace {

constexpr uint64_t kForestMagic = 0x7472657672466f72ull;
std::mutex g_forest_mu;
std::unordered_set<const trevr_forest*> g_forests;

enum : uint32_t { FERR_ACTIVE = 1u };   // backward's active set differs from the forward's

bool forest_live(const trevr_forest* f) {
  std::lock_guard<std::mutex> g(g_forest_mu);
  return f && g_forests.count(f) && f->magic == kForestMagic;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace layout: the device table, the error words, then each scene's
// tree workspace.
struct ForestLayout {
  size_t table, err;
  std::vector<size_t> tree_off, tree_bytes;
  size_t total;
};

trevr_status forest_layout(const trevr_params* params, int32_t S, const int64_t* offsets,
                           ForestLayout* L) {
  if (!params || !offsets) return set_error(TREVR_E_INVALID, "NULL params or offsets");
  if (S < 1) return set_error(TREVR_E_INVALID, "a forest needs at least one scene");
  if (offsets[0] != 0) return set_error(TREVR_E_INVALID, "offsets[0] must be 0");
  L->table = 0;
  L->err = align256(sizeof(DevTree) * (size_t)S);
  size_t o = align256(L->err + 16);
  L->tree_off.resize(S);
  L->tree_bytes.resize(S);
  for (int32_t s = 0; s < S; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    if (n <= 0) return set_error(TREVR_E_INVALID, "every scene needs at least one element");
    size_t tb = 0;
    const trevr_status rc = trevr_workspace_bytes(&params[s], n, &tb, nullptr);
    if (rc != TREVR_OK) return rc;
    L->tree_off[s] = o;
    L->tree_bytes[s] = tb;
    o = align256(o + tb);
  }
  L->total = o + 256;
  return TREVR_OK;
}

Launch forest_launch(const trevr_forest* f) {
  return Launch{f->stream, f->dtab, f->S, f->max_nodes, f->max_n, f->leaves_total,
                f->stack_large, f->cfg};
}

__global__ void k_zero_counters(const DevTree* __restrict__ TT) {
  const DevTree& T = TT[blockIdx.x];
  if (threadIdx.x < CNT_N) T.counters[threadIdx.x] = 0ull;
}

__global__ void k_hash_check(const unsigned long long* h, uint32_t* err) {
  if (threadIdx.x == 0 && h[0] != h[1]) atomicOr(err, FERR_ACTIVE);
}

// After an adjoint that reused the forward's state: when the active set did
// not match (FERR_ACTIVE), the gradients were computed for the wrong set,
// so every output is overwritten with NaN rather than left plausible.
__global__ void k_poison_if_stale(const uint32_t* err, double* gL, double* gk, int64_t nj,
                                  double* grho, int64_t n) {
  if (!(*err & FERR_ACTIVE)) return;
  const double nan = __longlong_as_double(0x7FF8000000000000ll);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nj;
       i += (int64_t)gridDim.x * blockDim.x) {
    gL[i] = nan;
    gk[i] = nan;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    grho[i] = nan;
}

#define TREVR_LAUNCH_CHECK(what)                                               \
  do {                                                                         \
    if ((rc = hip_check(hipGetLastError(), what)) != TREVR_OK) return rc;      \
  } while (0)

trevr_status zero_counters(const trevr_forest* f) {
  trevr_status rc;
  k_zero_counters<<<(unsigned)f->S, 64, 0, f->stream>>>(f->dtab);
  TREVR_LAUNCH_CHECK("k_zero_counters");
  return rc;
}

// Scratch of a batched call: the fixed part with room for every bucket's
// cut list, then the p-p lists, columns and pair depths of the plan; the
// adjoint adds the column adjoints, raw J and gradient accumulators.
struct ForestScratch {
  Scratch S;
  BwdArgs a;
  size_t gbeg, gbytes, fwd_end, bwd_end;
};

ForestScratch forest_carve(const trevr_forest* f, void* base) {
  ForestScratch fs{};
  fs.S = carve_scratch(base, f->leaves_total, (size_t)f->leaves_total * f->cut_cap);
  Carve dyn(base ? (char*)base + fs.S.fixed : nullptr);
  fs.S.nidx = dyn.take<uint32_t>(f->tot[TOT_NEAR]);
  fs.S.tpp = dyn.take<float>(f->tot[TOT_TPP]);
  fs.S.ptau = dyn.take<float>(f->tot[TOT_PTAU]);
  fs.fwd_end = fs.S.fixed + dyn.off + 256;
  fs.a.gtpp = dyn.take<float>(f->tot[TOT_TPP]);
  fs.a.jraw = dyn.take<double>(f->tot[TOT_JRAW]);
  fs.gbeg = align256(fs.S.fixed + dyn.off);
  Carve gcv(base ? (char*)base + fs.gbeg : nullptr);
  const GradDims dims{f->jn_total, f->n_total, f->nodes_total, f->nodesB_total, f->alpha_total,
                      f->leaves_total};
  fs.a.G = carve_grad(gcv, dims);
  fs.gbytes = align256(gcv.off);
  fs.bwd_end = fs.gbeg + fs.gbytes + 256;
  // the p-p job log: stream starts per bucket, the block counter, the blocks
  const uint64_t blocks = std::min<uint64_t>(f->job_log_bytes / (2ull * kLogBlock), 0xFFFFFF00ull);
  if (blocks > 0) {
    Carve lcv(base ? (char*)base + fs.bwd_end : nullptr);
    fs.S.jlog.tab = lcv.take<uint2>((size_t)4 * std::max<int64_t>(f->leaves_total, 1));
    fs.S.jlog.next = lcv.take<uint32_t>(64);
    fs.S.jlog.log = lcv.take<uint16_t>((size_t)blocks * kLogBlock);
    fs.S.jlog.blocks = (uint32_t)blocks;
    fs.bwd_end += align256(lcv.off) + 256;
  }
  return fs;
}

Items class_items(const Scratch& S, int B, int slot) {
  return Items{0u, 0xFFFFFFFFu, S.rng + 2 + 2 * (B - 1), S.q + 2 * slot};
}

// The forward's per-bucket work after the setup: p-p lists, walks of every
// active bucket, then per band count the p-p columns, p-p sources (J
// starts with them; J == nullptr: pair depths only) and the far field.
trevr_status forward_body(trevr_forest* f, const Scratch& S, const uint8_t* active,
                          const float* bg, double* J, bool far) {
  const Launch L = forest_launch(f);
  Prof* P = &f->prof;
  trevr_status rc;
  hipEvent_t e = prof_begin(P, L.st);
  if ((rc = near_fill(L, S)) != TREVR_OK) return rc;
  prof_end(P, L.st, TREVR_PROF_SETUP, e);
  e = prof_begin(P, L.st);
  if ((rc = walk_launch(L, S, Items{0u, 0xFFFFFFFFu, S.rng, nullptr},
                        (uint64_t)f->leaves_total, f->cut_cap)) != TREVR_OK)
    return rc;
  prof_end(P, L.st, TREVR_PROF_WALK, e);
  if (S.jlog.log && (rc = zero_words(L.st, S.jlog.next, 1)) != TREVR_OK) return rc;
  for (int B = 1; B <= kMaxBands; ++B) {
    const uint64_t cnt = (uint64_t)f->class_leaves[B - 1];
    if (cnt == 0) continue;
    e = prof_begin(P, L.st);
    if ((rc = launch_pp_rays(L, B, S, class_items(S, B, Q_PPR), cnt, active)) != TREVR_OK)
      return rc;
    prof_end(P, L.st, TREVR_PROF_NEAR, e);
    e = prof_begin(P, L.st);
    if ((rc = launch_pp_src(L, B, S, class_items(S, B, Q_PPS), cnt, active, J)) != TREVR_OK)
      return rc;
    const size_t recorded = P->pending.size();
    prof_end(P, L.st, TREVR_PROF_PP_SRC, e);
    if (P->pending.size() == recorded + 1)   // the same span in the near-field total
      P->pending.push_back({TREVR_PROF_NEAR, P->pending.back().second});
    e = prof_begin(P, L.st);
    if (far && (rc = launch_far(L, B, S, class_items(S, B, Q_FAR), cnt, f->cut_cap, bg, J,
                                active)) != TREVR_OK)
      return rc;
    prof_end(P, L.st, TREVR_PROF_REDUCE, e);
  }
  return TREVR_OK;
}

trevr_status batched_checks(trevr_forest* f, const float* bg, void* scratch, size_t bytes,
                            size_t need) {
  if (!f->planned) return set_error(TREVR_E_STATE, "plan the forest first (trevr_forest_plan)");
  if (!scratch) return set_error(TREVR_E_INVALID, "NULL scratch");
  if (f->any_bg && !bg) return set_error(TREVR_E_INVALID, "a scene with TREVR_BACKGROUND needs bg");
  if (bytes < need) return set_error(TREVR_E_CAPACITY, "scratch smaller than the forest's plan");
  return TREVR_OK;
}

// Launch configuration number k of the autotuner's candidates: bit 2 the
// bucket order (heaviest first / scene by scene), bit 1 the persistent grid
// (every resident slot / half of them), bit 0 the p-p culling granularity
// (kSub / kSub / 2 elements per box).
LaunchCfg config_of(int k) {
  LaunchCfg c;
  c.order = (k & 4) ? ORDER_SCENE : ORDER_COST;
  c.grid_div = (k & 2) ? 2u : 1u;
  c.pp_sub = (k & 1) ? kSub / 2 : kSub;
  return c;
}

}  // namespace

trevr_status forest_plan_impl(trevr_forest* f, void* scratch, size_t bytes) {
  const size_t cut_entries = default_cut_entries(f->leaves_total);
  Scratch S = carve_scratch(scratch, f->leaves_total, cut_entries);
  if (bytes < S.fixed) return set_error(TREVR_E_CAPACITY, "plan scratch too small");
  trevr_status rc;
  uint32_t* hb = f->host;
  uint32_t nb = 0, maxcut = 0;
  hipStream_t st = f->stream;
  for (;;) {
    const Launch L = forest_launch(f);
    if ((rc = zero_counters(f)) != TREVR_OK) return rc;
    if ((rc = setup_kernels(L, nullptr, S)) != TREVR_OK) return rc;
    hipError_t e = hipMemcpyAsync(hb, S.tot, TOT_N * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hb + 2 * TOT_N, S.rng + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hb + 2 * TOT_N + 1, S.ovf, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if ((rc = hip_check(e, "plan readback")) != TREVR_OK) return rc;
    std::memcpy(f->tot, hb, TOT_N * sizeof(uint64_t));
    nb = hb[2 * TOT_N];
    bool over = (hb[2 * TOT_N + 1] & OVF_SETUP) != 0u;
    maxcut = 0;
    // walks in batches of the plan's cut buffer; k_walk counts entries past
    // its capacity, so one pass gives the longest cut list
    for (uint32_t b0 = 0; b0 < nb && !over; b0 += kBatch) {
      const uint32_t cnt = std::min<uint32_t>(kBatch, nb - b0);
      if ((rc = walk_launch(L, S, Items{b0, b0 + cnt, nullptr, nullptr}, cnt,
                            kCutCap)) != TREVR_OK)
        return rc;
      e = hipMemcpyAsync(hb, S.ovf, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if ((rc = hip_check(e, "plan walk readback")) != TREVR_OK) return rc;
      over = (hb[0] & OVF_WALK) != 0u;
      maxcut = std::max(maxcut, hb[1]);
    }
    if (!over) break;
    if (f->stack_large)
      return set_error(TREVR_E_CAPACITY, "a traversal exceeds the large traversal stack");
    f->stack_large = true;
  }
  for (int k = 0; k < TOT_RECV; ++k)
    if (f->tot[k] > 0xFFFFFFFFull)
      return set_error(TREVR_E_CAPACITY, "the forest's p-p sizes exceed 32-bit offsets");
  f->cut_cap = (std::max<uint32_t>(maxcut, 1u) + 63u) & ~63u;
  f->planned = true;
  f->scratch_run = forest_carve(f, nullptr).bwd_end;
  f->fwd_scratch = nullptr;
  return TREVR_OK;
}

trevr_status forest_compute_impl(trevr_forest* f, const uint8_t* active, const float* bg,
                                 double* J, void* scratch) {
  ForestScratch fs = forest_carve(f, scratch);
  trevr_status rc;
  const uint64_t epoch = scratch_mark(scratch);
  f->fwd_scratch = nullptr;
  if ((rc = zero_counters(f)) != TREVR_OK) return rc;
  hipEvent_t e = prof_begin(&f->prof, f->stream);
  if ((rc = setup_kernels(forest_launch(f), active, fs.S)) != TREVR_OK) return rc;
  prof_end(&f->prof, f->stream, TREVR_PROF_SETUP, e);
  if ((rc = forward_body(f, fs.S, active, bg, J, true)) != TREVR_OK) return rc;
  for (trevr_tree* t : f->trees) t->counters_valid = true;
  f->fwd_scratch = scratch;
  f->fwd_epoch = epoch;
  return TREVR_OK;
}

trevr_status forest_backward_impl(trevr_forest* f, const uint8_t* active, const float* bg,
                                  const double* gJ, double* gL, double* gk, double* grho,
                                  void* scratch) {
  ForestScratch fs = forest_carve(f, scratch);
  const Scratch& S = fs.S;
  trevr_status rc;
  const bool reuse = f->fwd_scratch == scratch && scratch_unchanged(scratch, f->fwd_epoch);
  const uint64_t epoch = scratch_mark(scratch);
  f->fwd_scratch = nullptr;
  const Launch L = forest_launch(f);
  if ((rc = zero_words(f->stream, (char*)scratch + fs.gbeg, fs.gbytes / 4)) != TREVR_OK)
    return rc;
  if (reuse) {
    // the forward's state applies to the active set it was computed for
    if ((rc = launch_active_hash(L, active, S.ahash + 1)) != TREVR_OK) return rc;
    k_hash_check<<<1, 64, 0, f->stream>>>(S.ahash, f->ferr);
    TREVR_LAUNCH_CHECK("k_hash_check");
  } else {
    if ((rc = zero_counters(f)) != TREVR_OK) return rc;
    if ((rc = setup_kernels(L, active, S)) != TREVR_OK) return rc;
    if ((rc = forward_body(f, S, active, bg, nullptr, false)) != TREVR_OK) return rc;
  }
  BwdArgs a = fs.a;
  a.active = active;
  a.bg = bg;
  a.gJ = gJ;
  a.kept_tau = nullptr;
  a.kept_tex = nullptr;
  for (int B = 1; B <= kMaxBands; ++B) {
    const uint64_t cnt = (uint64_t)f->class_leaves[B - 1];
    if (cnt == 0) continue;
    if ((rc = bwd_items(L, B, S, a, class_items(S, B, 0), cnt, f->cut_cap, &f->prof)) !=
        TREVR_OK)
      return rc;
  }
  hipEvent_t e = prof_begin(&f->prof, f->stream);
  if ((rc = bwd_tree_pass(L, S, a.G, f->level_work, gL, gk, grho)) != TREVR_OK) return rc;
  prof_end(&f->prof, f->stream, TREVR_PROF_ADJ_TREE, e);
  if (reuse) {
    k_poison_if_stale<<<256, 256, 0, f->stream>>>(f->ferr, gL, gk, f->jn_total, grho,
                                                  f->n_total);
    TREVR_LAUNCH_CHECK("k_poison_if_stale");
  }
  f->fwd_scratch = scratch;
  f->fwd_epoch = epoch;
  return TREVR_OK;
}
#undef TREVR_LAUNCH_CHECK

}  // namespace trevr

using namespace trevr;

extern "C" {

trevr_status trevr_forest_workspace_bytes(const trevr_params* params, int32_t S,
                                          const int64_t* offsets, size_t* ws_bytes) {
  ForestLayout L;
  const trevr_status rc = forest_layout(params, S, offsets, &L);
  if (rc != TREVR_OK) return rc;
  if (ws_bytes) *ws_bytes = L.total;
  return TREVR_OK;
}

trevr_status trevr_forest_destroy(trevr_forest* f) {
  {
    std::lock_guard<std::mutex> g(g_forest_mu);
    if (!f || !g_forests.count(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
    g_forests.erase(f);
  }
  for (trevr_tree* t : f->trees)
    if (t) trevr_tree_destroy(t);
  if (f->host) (void)hipHostFree(f->host);
  prof_destroy(&f->prof);
  f->magic = 0;
  delete f;
  return TREVR_OK;
}

trevr_status trevr_build_forest(const trevr_params* params, int32_t S, const int64_t* offsets,
                                const float* x, const float* y, const float* z, const float* m,
                                const float* rho, const float* kappa, const float* lum, void* ws,
                                size_t ws_bytes, void* stream, trevr_forest** out) {
  if (!out) return set_error(TREVR_E_INVALID, "out is NULL");
  *out = nullptr;
  ForestLayout lay;
  trevr_status rc = forest_layout(params, S, offsets, &lay);
  if (rc != TREVR_OK) return rc;
  if (!x || !y || !z || !m || !rho || !kappa || !lum || !ws)
    return set_error(TREVR_E_INVALID, "NULL array argument");
  if (ws_bytes < lay.total) return set_error(TREVR_E_CAPACITY, "forest workspace too small");
  trevr_forest* f = new trevr_forest();
  f->magic = kForestMagic;
  f->S = S;
  f->params.assign(params, params + S);
  f->off.assign(offsets, offsets + S + 1);
  f->trees.assign(S, nullptr);
  f->stream = (hipStream_t)stream;
  f->ws = ws;
  f->ws_bytes = ws_bytes;
  f->dtab = (DevTree*)((char*)ws + lay.table);
  f->ferr = (uint32_t*)((char*)ws + lay.err);
  f->host = nullptr;
  f->planned = false;
  f->stack_large = false;
  f->cut_cap = kCutCap;
  f->scratch_run = 0;
  f->job_log_bytes = 0;
  f->fwd_scratch = nullptr;
  f->fwd_epoch = 0;
  f->cfg = LaunchCfg{};
  f->cfg_index = 0;
  std::memset(f->tot, 0, sizeof(f->tot));
  std::memset(f->class_leaves, 0, sizeof(f->class_leaves));
  {
    std::lock_guard<std::mutex> g(g_forest_mu);
    g_forests.insert(f);
  }
  rc = hip_check(hipHostMalloc((void**)&f->host, kHostWords * sizeof(uint32_t)), "hipHostMalloc");
  std::vector<DevTree> tab(S);
  int64_t koff = 0, boff = 0, noff = 0, lboff = 0, aoff = 0;
  f->n_total = f->jn_total = f->nodes_total = f->nodesB_total = f->alpha_total = 0;
  f->leaves_total = f->max_nodes = f->max_n = 0;
  f->any_bg = false;
  f->any_complex = false;
  for (int32_t s = 0; s < S && rc == TREVR_OK; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s], e0 = offsets[s];
    rc = trevr_build_tree(&params[s], n, x + e0, y + e0, z + e0, m + e0, rho + e0, kappa + koff,
                          lum + koff, (char*)ws + lay.tree_off[s], lay.tree_bytes[s], stream,
                          &f->trees[s]);
    if (rc != TREVR_OK) break;
    const trevr_tree* T = f->trees[s];
    DevTree D = T->dev;
    D.eoff = e0;
    D.joff = koff;
    D.boff = (int32_t)boff;
    D.noff = noff;
    D.lboff = lboff;
    D.aoff = aoff;
    tab[s] = D;
    koff += (int64_t)T->B * n;
    boff += T->B;
    noff += T->num_nodes;
    lboff += T->num_nodes * T->B;
    aoff += T->num_nodes * T->nclass * T->B;
    f->leaves_total += T->num_leaves;
    f->class_leaves[T->B - 1] += T->num_leaves;
    f->max_nodes = std::max<int64_t>(f->max_nodes, T->num_nodes);
    f->max_n = std::max<int64_t>(f->max_n, n);
    if (T->p.flags & TREVR_BACKGROUND) f->any_bg = true;
    if (T->p.flags & TREVR_COMPLEX_SRC) f->any_complex = true;
    for (size_t d = 0; d < T->levels.size(); ++d) {
      if (f->level_work.size() <= d) f->level_work.push_back(0);
      const int64_t w = (int64_t)(T->levels[d].second - T->levels[d].first) * T->nclass;
      f->level_work[d] = std::max(f->level_work[d], w);
    }
  }
  if (rc == TREVR_OK) {
    f->n_total = offsets[S];
    f->jn_total = koff;
    f->bands_total = (int32_t)boff;
    f->nodes_total = noff;
    f->nodesB_total = lboff;
    f->alpha_total = aoff;
    hipError_t e = hipMemcpyAsync(f->dtab, tab.data(), sizeof(DevTree) * (size_t)S,
                                  hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = hipMemsetAsync(f->ferr, 0, 16, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    rc = hip_check(e, "forest table upload");
  }
  if (rc != TREVR_OK) {
    const std::string msg = trevr_last_error();
    trevr_forest_destroy(f);
    return set_error(rc, msg);
  }
  *out = f;
  return TREVR_OK;
}

trevr_status trevr_forest_plan_bytes(const trevr_forest* f, size_t* bytes) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!bytes) return set_error(TREVR_E_INVALID, "NULL output");
  *bytes = carve_scratch(nullptr, f->leaves_total, default_cut_entries(f->leaves_total)).fixed;
  return TREVR_OK;
}

trevr_status trevr_forest_plan(trevr_forest* f, void* scratch, size_t scratch_bytes,
                               void* stream) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!scratch) return set_error(TREVR_E_INVALID, "NULL scratch");
  f->stream = (hipStream_t)stream;
  return forest_plan_impl(f, scratch, scratch_bytes);
}

trevr_status trevr_forest_scratch_bytes(const trevr_forest* f, size_t* bytes) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!bytes) return set_error(TREVR_E_INVALID, "NULL output");
  if (!f->planned) return set_error(TREVR_E_STATE, "plan the forest first (trevr_forest_plan)");
  *bytes = f->scratch_run;
  return TREVR_OK;
}

trevr_status trevr_forest_job_log(trevr_forest* f, size_t bytes) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  f->job_log_bytes = bytes;
  if (f->planned) f->scratch_run = forest_carve(f, nullptr).bwd_end;
  f->fwd_scratch = nullptr;
  return TREVR_OK;
}

trevr_status trevr_compute_J_batched(trevr_forest* f, const uint8_t* active, const float* bg,
                                     double* J, void* scratch, size_t scratch_bytes,
                                     void* stream) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!J) return set_error(TREVR_E_INVALID, "NULL J");
  trevr_status rc = batched_checks(f, bg, scratch, scratch_bytes, f->scratch_run);
  if (rc != TREVR_OK) return rc;
  f->stream = (hipStream_t)stream;
  return forest_compute_impl(f, active, bg, J, scratch);
}

trevr_status trevr_compute_J_backward_batched(trevr_forest* f, const uint8_t* active,
                                              const float* bg, const double* gJ, double* gL,
                                              double* gkappa, double* grho, void* scratch,
                                              size_t scratch_bytes, void* stream) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!gJ || !gL || !gkappa || !grho)
    return set_error(TREVR_E_INVALID, "NULL gradient pointer");
  if (f->any_complex)
    return set_error(TREVR_E_INVALID, "the adjoint does not cover the complex source model");
  trevr_status rc = batched_checks(f, bg, scratch, scratch_bytes, f->scratch_run);
  if (rc != TREVR_OK) return rc;
  f->stream = (hipStream_t)stream;
  return forest_backward_impl(f, active, bg, gJ, gL, gkappa, grho, scratch);
}

trevr_status trevr_forest_profile_enable(trevr_forest* f, int on) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  return prof_enable(&f->prof, f->stream, on != 0);
}

trevr_status trevr_forest_profile_read(trevr_forest* f, double* ms, int64_t* launches) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  return prof_read(&f->prof, f->stream, ms, launches);
}

trevr_status trevr_forest_check(trevr_forest* f) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  uint32_t fe = 0;
  hipError_t e = hipStreamSynchronize(f->stream);
  if (e == hipSuccess) e = hipMemcpy(&fe, f->ferr, sizeof(uint32_t), hipMemcpyDeviceToHost);
  trevr_status rc = hip_check(e, "forest error readback");
  if (rc != TREVR_OK) return rc;
  for (trevr_tree* t : f->trees) {
    t->stream = f->stream;
    if ((rc = trevr_check(t)) != TREVR_OK) return rc;
  }
  if (fe & FERR_ACTIVE)
    return set_error(TREVR_E_STATE,
                     "a batched backward ran on the forward state of a different active set");
  return TREVR_OK;
}

trevr_status trevr_forest_get_counters(trevr_forest* f, int32_t scene, trevr_counters* o) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!o) return set_error(TREVR_E_INVALID, "NULL output");
  if (scene >= f->S || scene < -1) return set_error(TREVR_E_INVALID, "scene out of range");
  if (scene >= 0) {
    f->trees[scene]->stream = f->stream;
    return trevr_get_counters(f->trees[scene], o);
  }
  std::memset(o, 0, sizeof(*o));
  for (trevr_tree* t : f->trees) {
    trevr_counters c;
    t->stream = f->stream;
    const trevr_status rc = trevr_get_counters(t, &c);
    if (rc != TREVR_OK) return rc;
    o->buckets += c.buckets;
    o->cells += c.cells;
    o->absorber_entries += c.absorber_entries;
    o->source_entries += c.source_entries;
    o->segments += c.segments;
    o->near_pairs += c.near_pairs;
    o->max_near = std::max(o->max_near, c.max_near);
    o->nodes += c.nodes;
    o->src_pairs += c.src_pairs;
    o->near_src_triples += c.near_src_triples;
    o->max_cut = std::max(o->max_cut, c.max_cut);
    o->max_stack = std::max(o->max_stack, c.max_stack);
    o->near_src_hits += c.near_src_hits;
    o->pp_log_entries += c.pp_log_entries;
  }
  return TREVR_OK;
}

trevr_status trevr_forest_set_config(trevr_forest* f, int32_t config) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (config < 0 || config >= TREVR_FOREST_CONFIGS)
    return set_error(TREVR_E_INVALID, "configuration out of range");
  f->cfg = config_of(config);
  f->cfg_index = config;
  return TREVR_OK;
}

trevr_status trevr_forest_get_config(const trevr_forest* f, int32_t* config) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!config) return set_error(TREVR_E_INVALID, "NULL output");
  *config = f->cfg_index;
  return TREVR_OK;
}

trevr_status trevr_forest_autotune(trevr_forest* f, const uint8_t* active, const float* bg,
                                   double* J, const double* gJ, double* gL, double* gkappa,
                                   double* grho, void* scratch, size_t scratch_bytes,
                                   void* stream, int32_t reps, double* times) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!J) return set_error(TREVR_E_INVALID, "NULL J");
  const bool adj = gJ != nullptr;
  if (adj && (!gL || !gkappa || !grho))
    return set_error(TREVR_E_INVALID, "NULL gradient pointer");
  trevr_status rc = batched_checks(f, bg, scratch, scratch_bytes, f->scratch_run);
  if (rc != TREVR_OK) return rc;
  f->stream = (hipStream_t)stream;
  reps = std::max(reps, 1);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if ((rc = hip_check(he, "hipEventCreate")) != TREVR_OK) return rc;
  int best = 0;
  float best_ms = 0.0f;
  for (int k = 0; k < TREVR_FOREST_CONFIGS && rc == TREVR_OK; ++k) {
    f->cfg = config_of(k);
    float ms = 0.0f;
    for (int r = 0; r <= reps && rc == TREVR_OK; ++r) {   // the first run warms up
      if (r == 1) he = hipEventRecord(e0, f->stream);
      rc = forest_compute_impl(f, active, bg, J, scratch);
      if (rc == TREVR_OK && adj)
        rc = forest_backward_impl(f, active, bg, gJ, gL, gkappa, grho, scratch);
    }
    if (rc != TREVR_OK) break;
    he = hipEventRecord(e1, f->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if ((rc = hip_check(he, "autotune timing")) != TREVR_OK) break;
    ms /= (float)reps;
    if (times) times[k] = ms;
    if (k == 0 || ms < best_ms) {
      best = k;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  f->cfg = config_of(best);
  f->cfg_index = best;
  return rc;
}

trevr_status trevr_forest_scene(trevr_forest* f, int32_t scene, trevr_tree** out) {
  if (!forest_live(f)) return set_error(TREVR_E_STATE, "unknown or destroyed forest");
  if (!out) return set_error(TREVR_E_INVALID, "NULL output");
  if (scene < 0 || scene >= f->S) return set_error(TREVR_E_INVALID, "scene out of range");
  *out = f->trees[scene];
  return TREVR_OK;
}

}  // extern "C"
