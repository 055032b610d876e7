// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "trevr_common.hpp"

namespace trevr {

// Traversal stacks live in LDS: the small one keeps the traversal kernels
// at 8 wavefronts per SIMD (the deepest stacks seen are a few hundred
// entries); a tree whose traversal overflows it switches to the large one.
constexpr int kStackSmall = 1024;
constexpr int kStackLarge = 8192;
constexpr uint32_t kCutCap = 2048;   // cut-list entries per bucket the buffer is sized for
constexpr size_t kStageCap = 4096;   // most staging words per bucket for the p-p set
constexpr uint32_t kNoRuns = 0xFFFFFFFFu;   // a staged p-p set that did not fit
// Staged runs (two words each after a two-word header) sorted in LDS: their
// count bound and the bits of a staging index in a sort key.
constexpr uint32_t kSortRuns = 2048;
constexpr int kSortIdxBits = 11;
static_assert((kStageCap - 2) / 2 <= kSortRuns && kSortRuns <= (1u << kSortIdxBits),
              "staged runs must fit the sort");

// Bump allocator over a caller-owned buffer (base == nullptr: size only).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T> T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Mutable device pointers of a tree (same memory the DevTree views).
struct TreeBufs {
  double* hdr;
  uint32_t* bbox_u;           // ordered-uint min/max of x, y, z
  uint64_t *keys, *keys_alt;
  uint32_t *vals, *vals_alt, *hist;
  float *x, *y, *z, *m, *rho, *kappa, *lum;
  double *h, *lbol;
  uint32_t* perm;
  uint32_t *b_first, *b_count, *b_c0, *b_c1, *b_size, *b_pre;
  int32_t *b_lown, *b_split;
  uint32_t* alloc;
  uint4* nk;
  uint2* nlink;
  uint32_t* next;
  double4 *cen, *sl;
  double *Lb, *kmass, *alpha64;
  float* alpha32;
  double* ray_n;
  int32_t* ray_class;
  int32_t* ray_anti;          // [nray] ray of the opposite direction
  double *csrc_d, *csrc_a;    // complex source model: [node][nray] lengths,
                              // [node][nray][B] absorption (null when off)
  double* geom;               // [64][nclass][3]: log w1, log w12, chord / L
  uint32_t* err;
  unsigned long long* counters;
  DevTree* dev;               // device copy of the tree's DevTree (one-scene table)
  uint2* levels;              // [kMaxLevels + 3] BFS index ranges per depth
};

struct SortCfg {
  static constexpr int kThreads = 256;
  static constexpr int kItems = 16;
  static constexpr int kTile = kThreads * kItems;
};

// Direction tables of an N_side: centres, classes (rays sharing |n_x|,
// |n_y|, |n_z| see the same transmission averages) and the combine
// geometry per prefix length and class.
struct DirTables {
  int nside = 0, nray = 0, nclass = 0;
  std::vector<double> ray_n;      // [nray][3]
  std::vector<int32_t> ray_class; // [nray]
  std::vector<int32_t> ray_anti;  // [nray] ray of the opposite direction
  std::vector<double> geom;       // [64][nclass][3]
};
DirTables make_dir_tables(int nside);

size_t layout_tree(const trevr_params& p, int64_t n, int nclass, void* base, TreeBufs* out);

}  // namespace trevr

// What the scratch holds after a compute_J (or a backward that redid the
// setup): bucket lists, p-p radii and lists, the cut lists of the last
// batch and the p-p columns for the active set with this fingerprint.
struct FwdState {
  bool valid;
  const void* scratch;
  uint64_t epoch;       // the library's write to that scratch that left it
  uint64_t hash;
  uint32_t nb;
  uint64_t near_total, tpp_total, ptau_total, jraw_total;
  bool cuts_kept;       // the cut buffer holds every bucket's cut list
  uint32_t cut_stride;  // ... at this many entries per bucket
  bool kept;            // far-source optical depths of the forward are in the scratch
};

namespace trevr {
// Kernel timing of a tree or a forest (trevr_profile_enable,
// trevr_forest_profile_enable): HIP event pairs recorded on the owner's
// stream around launches, folded into per-slot totals when read.
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[TREVR_PROF_SLOTS] = {};
  int64_t calls[TREVR_PROF_SLOTS] = {};
};
}  // namespace trevr

struct trevr_tree {
  uint64_t magic;
  trevr_params p;
  int64_t n;
  int32_t B, nray, nclass, depth;
  int64_t num_nodes, num_leaves;
  hipStream_t stream;
  void* ws;
  size_t ws_bytes;
  trevr::TreeBufs buf;
  trevr::DevTree dev;
  trevr::DirTables dirs;
  std::vector<std::pair<uint32_t, uint32_t>> levels;  // BFS index ranges per depth
  size_t scratch_needed;
  bool counters_valid;
  uint32_t* host_u32;                       // pinned readback buffer (kHostWords)
  FwdState fwd;
  bool stack_large;                         // traversals need the large LDS stack
  uint32_t cut_default;                     // cut-list entries per bucket to try first
  uint32_t stage_limit;                     // most staging words per bucket for p-p sets
  trevr::Prof prof;                         // kernel timing (trevr_profile_enable)
};

namespace trevr {
constexpr int kHostWords = 64;
// Copy the host DevTree of a tree (and its level table) to the device copy
// the kernels read; synchronises.
trevr_status upload_dev(trevr_tree* t);
trevr_status set_error(trevr_status s, const std::string& msg);
trevr_status hip_check(hipError_t e, const char* what);
trevr_status build_tree_impl(trevr_tree* t, const float* x, const float* y, const float* z,
                             const float* m, const float* rho, const float* kappa,
                             const float* lum);
trevr_status compute_J_impl(trevr_tree* t, const uint8_t* active, const float* bg, double* J,
                            void* scratch, size_t scratch_bytes);
trevr_status compute_J_backward_impl(trevr_tree* t, const uint8_t* active, const float* bg,
                                     const double* gJ, double* gL, double* gkappa, double* grho,
                                     void* scratch, size_t scratch_bytes);
size_t scratch_fixed_bytes(int64_t n);
// Every call that writes a scratch buffer takes a new epoch for it; a
// state recorded at epoch e is still in the buffer iff no call (on any
// tree) has written it since.
uint64_t scratch_mark(const void* scratch);
bool scratch_unchanged(const void* scratch, uint64_t epoch);
// Record an event pair on stream st around a phase (no-op unless profiling
// is on; p may be null).
hipEvent_t prof_begin(Prof* p, hipStream_t st);
void prof_end(Prof* p, hipStream_t st, int slot, hipEvent_t begin);
inline hipEvent_t prof_begin(trevr_tree* t) { return t ? prof_begin(&t->prof, t->stream) : nullptr; }
inline void prof_end(trevr_tree* t, int slot, hipEvent_t begin) {
  if (t) prof_end(&t->prof, t->stream, slot, begin);
}
// Start (clearing the totals) or stop recording; creates the event pool.
trevr_status prof_enable(Prof* p, hipStream_t st, bool on);
// Synchronise st and copy the totals out (any pointer may be null).
trevr_status prof_read(Prof* p, hipStream_t st, double* ms, int64_t* launches);
void prof_destroy(Prof* p);
}  // namespace trevr
