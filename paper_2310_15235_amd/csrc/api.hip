// C ABI of the library (declared in include/trevr2.h): parameter checks,
// workspace sizing, tree handles, counters, sticky errors and table export.

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>

#include "trevr_internal.hpp"

namespace trevr {

static thread_local std::string g_last_error;
static std::mutex g_reg_mu;
static std::unordered_set<const trevr_tree*> g_live;
constexpr uint64_t kMagic = 0x7472657672327472ull;

trevr_status set_error(trevr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

trevr_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return TREVR_OK;
  return set_error(TREVR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static bool live(const trevr_tree* t) {
  std::lock_guard<std::mutex> g(g_reg_mu);
  return t && g_live.count(t) && t->magic == kMagic;
}

static trevr_status check_params(const trevr_params* p, int64_t n) {
  if (!p) return set_error(TREVR_E_INVALID, "params is NULL");
  if (n <= 0 || n >= (int64_t)1 << 31) return set_error(TREVR_E_INVALID, "n must be in [1, 2^31)");
  const int ns = p->nside;
  if (ns < 1 || ns > kMaxNside || (ns & (ns - 1)))
    return set_error(TREVR_E_INVALID, "nside must be a power of two in [1, 16]");
  if (p->leaf_size < 1) return set_error(TREVR_E_INVALID, "leaf_size must be >= 1");
  if (p->n_bands < 1 || p->n_bands > kMaxBands)
    return set_error(TREVR_E_INVALID, "n_bands must be in [1, 16]");
  if (p->flags & ~(uint32_t)(TREVR_THICK_CORR | TREVR_NEAR_FIELD | TREVR_BACKGROUND |
                            TREVR_ABSORPTION_AVG | TREVR_DIRECTED | TREVR_KEEP_DEPTHS |
                            TREVR_COMPLEX_SRC))
    return set_error(TREVR_E_INVALID, "unknown flag bits");
  if (!(p->theta >= 0.0) || !std::isfinite(p->theta))
    return set_error(TREVR_E_INVALID, "theta must be finite and >= 0");
  if (!(p->rpp_min >= 0.0) || !std::isfinite(p->rpp_min))
    return set_error(TREVR_E_INVALID, "rpp_min must be finite and >= 0");
  if (p->box[3] > 0.0) {
    for (int a = 0; a < 4; ++a)
      if (!std::isfinite(p->box[a])) return set_error(TREVR_E_INVALID, "box must be finite");
  }
  if (p->flags & TREVR_DIRECTED) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->target[a]))
        return set_error(TREVR_E_INVALID, "TREVR_DIRECTED needs a finite target");
  }
  return TREVR_OK;
}

hipEvent_t prof_begin(Prof* p, hipStream_t st) {
  if (!p || !p->on || p->used + 2 > p->pool.size()) return nullptr;
  hipEvent_t e = p->pool[p->used++];
  if (hipEventRecord(e, st) != hipSuccess) return nullptr;
  return e;
}

void prof_end(Prof* p, hipStream_t st, int slot, hipEvent_t begin) {
  if (!p || !begin || p->used + 1 > p->pool.size()) return;
  hipEvent_t e = p->pool[p->used++];
  if (hipEventRecord(e, st) != hipSuccess) return;
  p->pending.push_back({slot, {begin, e}});
}

// Fold recorded event pairs into the totals (the stream is synchronised).
static void prof_collect(Prof* p) {
  for (auto& pe : p->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      p->ms[pe.first] += ms;
      p->calls[pe.first] += 1;
    }
  }
  p->pending.clear();
  p->used = 0;
}

trevr_status prof_enable(Prof* p, hipStream_t st, bool on) {
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_check(he, "sync");
  p->pending.clear();
  p->used = 0;
  for (int i = 0; i < TREVR_PROF_SLOTS; ++i) { p->ms[i] = 0.0; p->calls[i] = 0; }
  if (on && p->pool.empty()) {
    p->pool.resize(4096);
    for (auto& e : p->pool) {
      he = hipEventCreate(&e);
      if (he != hipSuccess) return hip_check(he, "hipEventCreate");
    }
  }
  p->on = on;
  return TREVR_OK;
}

trevr_status prof_read(Prof* p, hipStream_t st, double* ms, int64_t* launches) {
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_check(he, "sync");
  prof_collect(p);
  for (int i = 0; i < TREVR_PROF_SLOTS; ++i) {
    if (ms) ms[i] = p->ms[i];
    if (launches) launches[i] = p->calls[i];
  }
  return TREVR_OK;
}

void prof_destroy(Prof* p) {
  for (auto& e : p->pool) (void)hipEventDestroy(e);
  p->pool.clear();
}

trevr_status upload_dev(trevr_tree* t) {
  t->dev.depth = (int32_t)t->levels.size();
  hipError_t e = hipMemcpyAsync(t->buf.dev, &t->dev, sizeof(DevTree), hipMemcpyHostToDevice,
                                t->stream);
  if (e == hipSuccess && !t->levels.empty())
    e = hipMemcpyAsync(t->buf.levels, t->levels.data(), t->levels.size() * sizeof(uint2),
                       hipMemcpyHostToDevice, t->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
  return hip_check(e, "tree table upload");
}

}  // namespace trevr

using namespace trevr;

extern "C" {

const char* trevr_status_string(trevr_status s) {
  switch (s) {
    case TREVR_OK: return "ok";
    case TREVR_E_INVALID: return "invalid argument";
    case TREVR_E_CAPACITY: return "workspace or scratch too small";
    case TREVR_E_HIP: return "HIP runtime error";
    case TREVR_E_STATE: return "unknown or destroyed tree handle";
    case TREVR_E_DATA: return "invalid input data";
  }
  return "unknown status";
}

const char* trevr_last_error(void) { return g_last_error.c_str(); }

trevr_status trevr_profile_enable(trevr_tree* t, int on) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  return prof_enable(&t->prof, t->stream, on != 0);
}

trevr_status trevr_profile_read(trevr_tree* t, double* ms, int64_t* launches) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  return prof_read(&t->prof, t->stream, ms, launches);
}

trevr_status trevr_workspace_bytes(const trevr_params* p, int64_t n, size_t* tree_bytes,
                                   size_t* scratch_bytes) {
  trevr_status rc = check_params(p, n);
  if (rc != TREVR_OK) return rc;
  const DirTables d = make_dir_tables(p->nside);
  if (tree_bytes) *tree_bytes = layout_tree(*p, n, d.nclass, nullptr, nullptr);
  if (scratch_bytes) *scratch_bytes = scratch_fixed_bytes(n) + sizeof(uint32_t) * 64 * (size_t)n + 512;
  return TREVR_OK;
}

trevr_status trevr_build_tree(const trevr_params* p, int64_t n, const float* x, const float* y,
                              const float* z, const float* m, const float* rho,
                              const float* kappa, const float* lum, void* tree_ws,
                              size_t tree_ws_bytes, void* stream, trevr_tree** out) {
  trevr_status rc = check_params(p, n);
  if (rc != TREVR_OK) return rc;
  if (!out) return set_error(TREVR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!x || !y || !z || !m || !rho || !kappa || !lum || !tree_ws)
    return set_error(TREVR_E_INVALID, "NULL array argument");
  trevr_tree* T = new trevr_tree();
  T->magic = kMagic;
  T->p = *p;
  T->n = n;
  T->B = p->n_bands;
  T->dirs = make_dir_tables(p->nside);
  T->nray = T->dirs.nray;
  T->nclass = T->dirs.nclass;
  T->stream = (hipStream_t)stream;
  T->ws = tree_ws;
  T->ws_bytes = tree_ws_bytes;
  T->scratch_needed = 0;
  T->counters_valid = false;
  T->host_u32 = nullptr;
  T->fwd = FwdState{false, nullptr, 0, 0, 0, 0, 0, 0, 0, false, 0, false};
  T->stack_large = false;
  T->cut_default = kCutCap;
  T->stage_limit = (uint32_t)kStageCap;
  const size_t need = layout_tree(*p, n, T->nclass, nullptr, nullptr);
  if (tree_ws_bytes < need) {
    delete T;
    return set_error(TREVR_E_CAPACITY, "tree workspace too small");
  }
  layout_tree(*p, n, T->nclass, tree_ws, &T->buf);
  DevTree& D = T->dev;
  const TreeBufs& b = T->buf;
  D.n = n;
  D.B = T->B;
  D.nside = p->nside;
  D.nray = T->nray;
  D.nclass = T->nclass;
  D.leaf_size = p->leaf_size;
  D.flags = p->flags;
  D.theta2 = p->theta * p->theta;
  D.rpp_min = p->rpp_min;
  D.wbeam = 2.0 * std::tan(std::acos(1.0 - 2.0 / T->nray));
  for (int a = 0; a < 3; ++a) D.target[a] = p->target[a];
  D.stack_limit = kStackSmall;
  D.hdr = b.hdr;
  D.x = b.x; D.y = b.y; D.z = b.z; D.m = b.m; D.rho = b.rho;
  D.h = b.h; D.lbol = b.lbol; D.kappa = b.kappa; D.lum = b.lum; D.perm = b.perm;
  D.nk = b.nk; D.nlink = b.nlink; D.next = b.next; D.cen = b.cen; D.Lb = b.Lb;
  D.alpha = b.alpha32; D.ray_n = b.ray_n; D.ray_class = b.ray_class;
  D.ray_anti = b.ray_anti; D.csrc_d = b.csrc_d; D.csrc_a = b.csrc_a;
  D.err = b.err; D.counters = b.counters;
  D.b_pre = b.b_pre; D.b_lown = b.b_lown; D.b_split = b.b_split;
  D.alpha64 = b.alpha64; D.geom = b.geom; D.levels = b.levels;
  D.boff = 0; D.eoff = 0; D.joff = 0; D.noff = 0; D.lboff = 0; D.aoff = 0;
  {
    std::lock_guard<std::mutex> g(g_reg_mu);
    g_live.insert(T);
  }
  rc = hip_check(hipHostMalloc((void**)&T->host_u32, kHostWords * sizeof(uint32_t)), "hipHostMalloc");
  if (rc == TREVR_OK) rc = build_tree_impl(T, x, y, z, m, rho, kappa, lum);
  if (rc != TREVR_OK) {
    trevr_tree_destroy(T);
    return rc;
  }
  D.num_nodes = T->num_nodes;
  if ((rc = upload_dev(T)) != TREVR_OK) {
    trevr_tree_destroy(T);
    return rc;
  }
  *out = T;
  return TREVR_OK;
}

trevr_status trevr_compute_J(trevr_tree* t, const uint8_t* active, const float* bg, double* J,
                             void* scratch, size_t scratch_bytes, void* stream) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (!J || !scratch) return set_error(TREVR_E_INVALID, "NULL J or scratch");
  if ((t->p.flags & TREVR_BACKGROUND) && !bg)
    return set_error(TREVR_E_INVALID, "TREVR_BACKGROUND needs bg");
  t->stream = (hipStream_t)stream;
  return compute_J_impl(t, active, bg, J, scratch, scratch_bytes);
}

// Scratch of trevr_compute_J_noalloc: a fixed device array, one copy per GPU.
// Host code never passes the array's name to the device: its device address
// on each GPU is looked up once (hipGetSymbolAddress, with that GPU current)
// and kept in g_noalloc_ptr.
static __device__ __align__(256) unsigned char noalloc_scratch[TREVR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kMaxDevices] = {};

static trevr_status noalloc_scratch_ptr(void** out) {
  int dev = -1;
  trevr_status rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (rc != TREVR_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(TREVR_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)), "hipGetSymbolAddress");
    if (rc != TREVR_OK) return rc;
    if (!p) return set_error(TREVR_E_HIP, "no device address for the fixed scratch array");
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return TREVR_OK;
}

trevr_status trevr_compute_J_noalloc(trevr_tree* t, const uint8_t* active, const float* bg,
                                     double* J, void* stream) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (!J) return set_error(TREVR_E_INVALID, "NULL J");
  if ((t->p.flags & TREVR_BACKGROUND) && !bg)
    return set_error(TREVR_E_INVALID, "TREVR_BACKGROUND needs bg");
  void* ptr = nullptr;
  trevr_status rc = noalloc_scratch_ptr(&ptr);
  if (rc != TREVR_OK) return rc;
  t->stream = (hipStream_t)stream;
  rc = compute_J_impl(t, active, bg, J, ptr, TREVR_NOALLOC_SCRATCH_BYTES);
  if (rc == TREVR_E_CAPACITY) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "compute_J_noalloc: this call needs %zu bytes of scratch, more than the fixed "
                  "%zu-byte device array",
                  t->scratch_needed, (size_t)TREVR_NOALLOC_SCRATCH_BYTES);
    return set_error(TREVR_E_CAPACITY, msg);
  }
  return rc;
}

trevr_status trevr_compute_J_backward(trevr_tree* t, const uint8_t* active, const float* bg,
                                      const double* gJ, double* gL, double* gkappa,
                                      double* grho, void* scratch, size_t scratch_bytes,
                                      void* stream) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (!gJ || !gL || !gkappa || !grho || !scratch)
    return set_error(TREVR_E_INVALID, "NULL gradient or scratch pointer");
  if (t->p.flags & TREVR_COMPLEX_SRC)
    return set_error(TREVR_E_INVALID, "the adjoint does not cover the complex source model");
  if ((t->p.flags & TREVR_BACKGROUND) && !bg)
    return set_error(TREVR_E_INVALID, "TREVR_BACKGROUND needs bg");
  t->stream = (hipStream_t)stream;
  return compute_J_backward_impl(t, active, bg, gJ, gL, gkappa, grho, scratch, scratch_bytes);
}

trevr_status trevr_tree_tune(trevr_tree* t, int key, int64_t value) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  switch (key) {
    case TREVR_TUNE_STACK:
      if (value < 64 || value > kStackSmall)
        return set_error(TREVR_E_INVALID, "stack limit must be in [64, 1024]");
      t->dev.stack_limit = (int32_t)value;
      t->stack_large = false;
      return hip_check(hipDeviceSynchronize() == hipSuccess
                           ? hipMemcpy(t->buf.dev, &t->dev, sizeof(DevTree), hipMemcpyHostToDevice)
                           : hipErrorUnknown,
                       "tree table upload");
    case TREVR_TUNE_CUT:
      if (value < 64 || value > (int64_t)kCutCap)
        return set_error(TREVR_E_INVALID, "cut-list length must be in [64, 2048]");
      t->cut_default = (uint32_t)value;
      return TREVR_OK;
    case TREVR_TUNE_STAGE:
      if (value < 0 || value > (int64_t)kStageCap)
        return set_error(TREVR_E_INVALID, "staging words must be in [0, 4096]");
      t->stage_limit = (uint32_t)value;
      return TREVR_OK;
    default:
      return set_error(TREVR_E_INVALID, "unknown tuning key");
  }
}

trevr_status trevr_scratch_needed(const trevr_tree* t, size_t* bytes) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (!bytes) return set_error(TREVR_E_INVALID, "NULL output");
  *bytes = t->scratch_needed;
  return TREVR_OK;
}

static trevr_status read_err(trevr_tree* t) {
  uint32_t e = 0;
  hipError_t he = hipStreamSynchronize(t->stream);
  if (he == hipSuccess) he = hipMemcpy(&e, t->buf.err, sizeof(uint32_t), hipMemcpyDeviceToHost);
  trevr_status rc = hip_check(he, "error readback");
  if (rc != TREVR_OK) return rc;
  if (e & ERR_DATA) return set_error(TREVR_E_DATA, "non-positive or non-finite element data");
  return TREVR_OK;
}

trevr_status trevr_check(trevr_tree* t) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  return read_err(t);
}

trevr_status trevr_get_counters(trevr_tree* t, trevr_counters* o) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (!o) return set_error(TREVR_E_INVALID, "NULL output");
  unsigned long long c[CNT_N];
  hipError_t he = hipStreamSynchronize(t->stream);
  if (he == hipSuccess) he = hipMemcpy(c, t->buf.counters, sizeof(c), hipMemcpyDeviceToHost);
  trevr_status rc = hip_check(he, "counter readback");
  if (rc != TREVR_OK) return rc;
  if (!t->counters_valid) std::memset(c, 0, sizeof(c));
  o->buckets = (int64_t)c[CNT_BUCKETS];
  o->cells = (int64_t)c[CNT_CELLS];
  o->absorber_entries = (int64_t)c[CNT_ABS];
  o->source_entries = (int64_t)c[CNT_SRC];
  o->segments = (int64_t)c[CNT_SEG];
  o->near_pairs = (int64_t)c[CNT_NEAR_PAIRS];
  o->max_near = (int64_t)c[CNT_MAX_NEAR];
  o->nodes = t->num_nodes;
  o->src_pairs = (int64_t)c[CNT_SRC_PAIRS];
  o->near_src_triples = (int64_t)c[CNT_NS_TRIPLES];
  o->max_cut = (int64_t)c[CNT_MAX_CUT];
  o->max_stack = (int64_t)c[CNT_MAX_STACK];
  o->near_src_hits = (int64_t)c[CNT_NS_HITS];
  o->pp_log_entries = (int64_t)c[CNT_PP_LOG];
  return TREVR_OK;
}

trevr_status trevr_tree_destroy(trevr_tree* t) {
  {
    std::lock_guard<std::mutex> g(g_reg_mu);
    if (!t || !g_live.count(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
    g_live.erase(t);
  }
  t->magic = 0;
  (void)hipStreamSynchronize(t->stream);
  prof_destroy(&t->prof);
  if (t->host_u32) (void)hipHostFree(t->host_u32);
  delete t;
  return TREVR_OK;
}

trevr_status trevr_tree_info(const trevr_tree* t, int64_t* num_nodes, int32_t* num_classes,
                             int32_t* depth, double* root_box) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  if (num_nodes) *num_nodes = t->num_nodes;
  if (num_classes) *num_classes = t->nclass;
  if (depth) *depth = t->depth;
  if (root_box) {
    hipError_t he = hipStreamSynchronize(t->stream);
    if (he == hipSuccess) he = hipMemcpy(root_box, t->buf.hdr, 4 * sizeof(double), hipMemcpyDeviceToHost);
    return hip_check(he, "root box readback");
  }
  return TREVR_OK;
}

trevr_status trevr_tree_export(trevr_tree* t, int64_t* perm, int64_t* ints, double* box,
                               double* cen, double* Lb, double* Lbol, float* alpha,
                               int32_t* ray_class, double* kmass, double* csrc_d,
                               double* csrc_a) {
  if (!live(t)) return set_error(TREVR_E_STATE, "unknown or destroyed tree handle");
  hipError_t he = hipStreamSynchronize(t->stream);
  if (he != hipSuccess) return hip_check(he, "sync");
  const int64_t nn = t->num_nodes, n = t->n;
  const int B = t->B, C = t->nclass;
  auto dl = [&](void* dst, const void* src, size_t bytes) -> bool {
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
  };
  bool ok = true;
  if (perm) {
    std::vector<uint32_t> p32(n);
    ok = ok && dl(p32.data(), t->buf.perm, sizeof(uint32_t) * n);
    for (int64_t i = 0; i < n; ++i) perm[i] = p32[i];
  }
  if (ints || box) {
    std::vector<uint32_t> first(nn), count(nn), c0(nn), c1(nn), size(nn), pre(nn);
    std::vector<int32_t> lown(nn), split(nn);
    std::vector<uint4> nk(nn);
    double hdr[8];
    ok = ok && dl(first.data(), t->buf.b_first, 4 * nn) && dl(count.data(), t->buf.b_count, 4 * nn) &&
         dl(c0.data(), t->buf.b_c0, 4 * nn) && dl(c1.data(), t->buf.b_c1, 4 * nn) &&
         dl(size.data(), t->buf.b_size, 4 * nn) && dl(pre.data(), t->buf.b_pre, 4 * nn) &&
         dl(lown.data(), t->buf.b_lown, 4 * nn) && dl(split.data(), t->buf.b_split, 4 * nn) &&
         dl(nk.data(), t->buf.nk, sizeof(uint4) * nn) && dl(hdr, t->buf.hdr, sizeof(hdr));
    if (ok) {
      for (int64_t i = 0; i < nn; ++i) {
        const int64_t p = pre[i];
        const bool leaf = split[i] < 0;
        if (ints) {
          int64_t* o = ints + 7 * p;
          o[0] = first[i];
          o[1] = count[i];
          o[2] = lown[i];
          o[3] = split[i];
          o[4] = leaf ? -1 : (int64_t)pre[c0[i]];
          o[5] = leaf ? -1 : (int64_t)pre[c1[i]];
          o[6] = p + size[i];
        }
        if (box) {
          const uint4 k = nk[p];
          const int l = (int)(k.w & 63u);
          const uint32_t kk[3] = {k.x, k.y, k.z};
          for (int a = 0; a < 3; ++a) {
            const double side = std::ldexp(hdr[3], -nbits_axis(l, a));
            box[6 * p + a] = hdr[a] + (double)kk[a] * side;
            box[6 * p + 3 + a] = hdr[a] + (double)(kk[a] + 1u) * side;
          }
        }
      }
    }
  }
  if (cen || Lbol) {
    std::vector<double4> cv(nn);
    ok = ok && dl(cv.data(), t->buf.cen, sizeof(double4) * nn);
    for (int64_t i = 0; ok && i < nn; ++i) {
      if (cen) { cen[3 * i] = cv[i].x; cen[3 * i + 1] = cv[i].y; cen[3 * i + 2] = cv[i].z; }
      if (Lbol) Lbol[i] = cv[i].w;
    }
  }
  if (Lb) ok = ok && dl(Lb, t->buf.Lb, sizeof(double) * nn * B);
  if (alpha) ok = ok && dl(alpha, t->buf.alpha32, sizeof(float) * nn * C * B);
  if (ray_class) std::memcpy(ray_class, t->dirs.ray_class.data(), sizeof(int32_t) * t->nray);
  if (kmass) ok = ok && dl(kmass, t->buf.kmass, sizeof(double) * nn);
  if ((csrc_d || csrc_a) && !t->buf.csrc_d)
    return set_error(TREVR_E_STATE, "the tree has no complex source tables");
  if (csrc_d) ok = ok && dl(csrc_d, t->buf.csrc_d, sizeof(double) * nn * t->nray);
  if (csrc_a) ok = ok && dl(csrc_a, t->buf.csrc_a, sizeof(double) * nn * t->nray * B);
  if (!ok) return set_error(TREVR_E_HIP, "export copy failed");
  return TREVR_OK;
}

}  // extern "C"
