// Host-side pieces of the mean intensity path shared by the forward
// (compute_j.hip), the adjoint (compute_j_bwd.hip) and the batched forest
// (forest.hip): the scratch layout of the per-bucket arrays and the launches
// that run unchanged for one tree or for the scenes of a forest.
#pragma once

#include <functional>
#include <vector>

#include "trevr_internal.hpp"
#include "path_device.hpp"

namespace trevr {

// Per-compute scratch.  A fixed part sized by the number of leaves (bucket
// arrays in processing order and in discovery order, cost bins, work-queue
// counters, the cut lists of one batch), then a dynamic part sized by the
// bucket setup: p-p lists, p-p optical depths per (receiver, ray, band),
// pair optical depths per (receiver, luminous p-p element, band) and the
// far-source depths kept for the adjoint.
struct Scratch {
  // zeroed at the start of every call (one contiguous run of words)
  uint32_t* rng;                // {0, buckets}, then [begin, end) per band count
  uint32_t* q;                  // work-queue counter pairs, Q_N of them
  unsigned long long* tot;      // 64-bit totals of the dynamic sizes (k_reorder)
  uint32_t* ovf;                // overflow bits, largest cut of a walk
  unsigned long long* ahash;    // [2] active-set fingerprints
  uint32_t* bins;               // cost bins per band count
  uint32_t *ncnt, *tcnt, *jcnt, *pcnt;   // sizes, scanned in place into offsets
  size_t zero_words;            // words from rng to the end of pcnt
  // processing order
  uint32_t *blist, *bscene, *bnact, *nlumc, *bstat;
  double *brad, *bprev;         // p-p radius; before its last growth (-1: none)
  uint32_t* barg;               // element that set the radius by that growth
  uint32_t* bsrc;               // discovery index of each bucket
  // discovery order
  uint32_t *blist_raw, *bscene_raw, *bnact_raw, *ncnt_raw, *nlumc_raw, *bbin, *barg_raw;
  double *brad_raw, *bprev_raw;
  uint2* cut;
  size_t cut_entries;           // capacity of the cut-list buffer
  // the p-p sets the bucket setup found, stage_cap words per bucket (a
  // multiple of 64; 0: none) in discovery order; they live in the cut-list
  // buffer, which holds nothing between the setup and the p-p lists
  uint32_t* stage;
  uint32_t stage_cap;
  // dynamic part
  uint32_t* nidx;
  float* tpp;
  float* ptau;                  // optical depth per (receiver, p-p source) pair and band
  float *kept_tau, *kept_tex;   // far-source optical depths kept for the adjoint (or null)
  JobLog jlog;                  // p-p job log of a forest (log null: none)
  size_t fixed;                 // bytes of the fixed part
};

// Slots of tot.
enum { TOT_NEAR = 0, TOT_TPP, TOT_PTAU, TOT_JRAW, TOT_RECV, TOT_N = 8 };

Scratch carve_scratch(void* base, int64_t leaves, size_t cut_entries);
// Default cut-list capacity of a lone tree's scratch.
size_t default_cut_entries(int64_t leaves);

// Where the launches of a call run: the device table of trees (one per
// scene), the largest tree (for grids over nodes and elements) and the
// number of leaves of all scenes (no call has more buckets).
// Launch options that change speed, never results beyond FP32 rounding of
// atomic sums: bucket order, persistent workgroups per CU (all that fit,
// divided by grid_div) and the p-p culling granularity (kSub or kSub / 2).
struct LaunchCfg {
  uint32_t order = ORDER_COST;
  uint32_t grid_div = 1;
  int pp_sub = kSub;
};

struct Launch {
  hipStream_t st;
  const DevTree* TT;
  int S;
  int64_t max_nodes, max_n;
  int64_t leaves;
  bool stack_large;
  LaunchCfg cfg;
};
Launch tree_launch(const trevr_tree* T);

// Workgroups of a persistent launch of `fn` (threads each): as many as are
// resident on the device at once (divided by div), at most `items`, at
// least 1.
unsigned persistent_grid(const void* fn, int threads, uint64_t items, uint32_t div);

trevr_status zero_words(hipStream_t st, void* p, size_t words);

// Bucket setup without synchronising: active buckets of every scene, p-p
// radii and set sizes, grouping by band count and heaviest-first order,
// per-bucket offsets of the dynamic scratch and their 64-bit totals, the
// active-set fingerprint in ahash[0].
trevr_status setup_kernels(const Launch& L, const uint8_t* active, const Scratch& S);
// Fingerprint of the active set of every scene into *out (zeroed first).
trevr_status launch_active_hash(const Launch& L, const uint8_t* active,
                                unsigned long long* out);
// Fill the p-p lists (S.nidx must be set).
trevr_status near_fill(const Launch& L, const Scratch& S);
// Tree walks of the items into the cut lists (cap entries each).
trevr_status walk_launch(const Launch& L, const Scratch& S, const Items& I, uint64_t count,
                         uint32_t cap);
// p-p columns per (receiver, ray, band) and, for the sources, pair optical
// depths and (with J) the p-p part of J, of the items of band count B.
trevr_status launch_pp_rays(const Launch& L, int B, const Scratch& S, const Items& I,
                            uint64_t count, const uint8_t* active);
trevr_status launch_pp_src(const Launch& L, int B, const Scratch& S, const Items& I,
                           uint64_t count, const uint8_t* active, double* J);
// The far field of the items of band count B (J already holds their p-p part).
trevr_status launch_far(const Launch& L, int B, const Scratch& S, const Items& I,
                        uint64_t count, uint32_t cap, const float* bg, double* J,
                        const uint8_t* active);

// Lone-tree helpers (synchronising): the setup with its readback and the
// stack retry; the walks of a batch with the cut-list retry.
trevr_status bucket_setup(trevr_tree* T, const uint8_t* active, Scratch& S, uint32_t* nb,
                          uint64_t tot[TOT_N], uint64_t* hash);
trevr_status active_hash(trevr_tree* T, const uint8_t* active, unsigned long long* dev_slot,
                         uint64_t* hash);
// Places kept_tau / kept_tex (after the p-p part of the dynamic region).
void take_kept(const trevr_tree* T, Scratch& S, Carve& cv, uint32_t nb);
// Tree walks of buckets [b0, b0 + cnt) into the cut lists, cut_default
// entries per bucket; then run(s0, scnt, cap) for the buckets whose cut
// lists are ready (stride cap).  Synchronises once.  A batch whose walks
// ran out of the traversal stack is walked again with the large stack; one
// where a bucket needs more entries again in parts with room for the
// longest (*whole = false).
trevr_status walk_batch(trevr_tree* T, const Scratch& S, uint32_t b0, uint32_t cnt,
                        const std::function<trevr_status(uint32_t, uint32_t, uint32_t)>& run,
                        bool* whole);
// Sizes of the gradient accumulators (sums over the scenes of a forest).
struct GradDims {
  int64_t jn;       // sum of B n
  int64_t n;        // elements
  int64_t nodes;
  int64_t nodesB;   // sum of nodes x B
  int64_t alpha;    // sum of nodes x classes x B
  int64_t leaves;
};

Grad carve_grad(Carve& cv, const GradDims& d);
// The adjoint's per-bucket kernels (p-p sources, far field, p-p columns) for
// the items of band count B; prof (nullable) records their times.
trevr_status bwd_items(const Launch& L, int B, const Scratch& S, const BwdArgs& a,
                       const Items& I, uint64_t count, uint32_t cap, Prof* prof);
// After the per-bucket kernels: r_pp adjoints, sums of the accumulator
// copies, the tree top-down per depth (level_work[d]: the widest scene's
// (nodes x classes) at depth d) and the gradients in input order.
trevr_status bwd_tree_pass(const Launch& L, const Scratch& S, const Grad& G,
                           const std::vector<int64_t>& level_work, double* gL, double* gk,
                           double* grho);

inline Items host_items(const Scratch& S, int slot, uint32_t b0, uint32_t cnt) {
  return Items{b0, b0 + cnt, nullptr, S.q + 2 * slot};
}

}  // namespace trevr
