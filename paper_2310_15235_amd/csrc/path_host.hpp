// Host-side pieces of the mean intensity path shared by the forward
// (compute_j.hip) and the adjoint (compute_j_bwd.hip): the scratch layout of
// the per-bucket arrays and the launches both run unchanged.
#pragma once

#include <functional>

#include "trevr_internal.hpp"

namespace trevr {

// Per-compute scratch: per-bucket arrays in processing order (and in
// discovery order, before the cost reordering), cost bins, cut lists of one
// batch; then, sized after the
// bucket readback, the p-p lists and the p-p optical depths per
// (receiver, ray, band).
struct Scratch {
  uint32_t *blist, *bnact, *ncnt, *pcnt, *nlumc, *bstat, *nb, *ovf;
  double *brad, *bprev;         // p-p radius; before its last growth (-1: none)
  unsigned long long* ahash;    // [2] active-set fingerprints
  uint32_t *blist_raw, *bnact_raw, *ncnt_raw, *nlumc_raw;
  double *brad_raw, *bprev_raw;
  uint32_t *bbin, *bins;
  uint2* cut;
  size_t cut_entries;           // capacity of the cut-list buffer
  uint32_t* nidx;
  float* tpp;
  float* ptau;                  // optical depth per (receiver, p-p source) pair
  float *kept_tau, *kept_tex;   // far-source optical depths kept for the adjoint (or null)
  size_t fixed;     // bytes of the part above (before the p-p lists)
};

Scratch carve_scratch(void* base, int64_t nleaves);
// Places kept_tau / kept_tex (after the p-p part of the dynamic region).
void take_kept(const trevr_tree* T, Scratch& S, Carve& cv, uint32_t nb);

// Active buckets, p-p radii and set sizes, heaviest-first order, offsets of
// the p-p lists (ncnt), the receivers (bnact) and the (receiver, p-p
// source) pairs (pcnt); reads back counts = {buckets, p-p entries, active
// receivers, pairs} and the active-set fingerprint (synchronises).
trevr_status bucket_setup(trevr_tree* T, const uint8_t* active, Scratch& S, uint32_t counts[4],
                          uint64_t* hash);
// Fingerprint of the active set alone, computed in dev_slot (synchronises).
trevr_status active_hash(trevr_tree* T, const uint8_t* active, unsigned long long* dev_slot,
                         uint64_t* hash);
// Fill the p-p lists (S.nidx must be set).
trevr_status near_fill(trevr_tree* T, const Scratch& S, uint32_t nb);
// Tree walks of buckets [b0, b0 + cnt) into the cut lists, kCutCap entries
// per bucket; then run(s0, scnt, cap) for the buckets whose cut lists are
// ready (stride cap).  Synchronises once.  A batch whose walks ran out of
// the traversal stack is walked again with the large stack; one where a
// bucket needs more than kCutCap entries again in parts with room for the
// longest (*whole = false).
trevr_status walk_batch(trevr_tree* T, const Scratch& S, uint32_t b0, uint32_t cnt, uint32_t nb,
                        const std::function<trevr_status(uint32_t, uint32_t, uint32_t)>& run,
                        bool* whole);
// p-p optical depth per (receiver, ray, band) of buckets [b0, b0 + cnt) into S.tpp.
trevr_status launch_pp_rays(trevr_tree* T, const Scratch& S, uint32_t b0, uint32_t nb,
                            uint32_t cnt, const uint8_t* active);
// p-p sources of buckets [b0, b0 + cnt): the pair optical depths into
// S.ptau and, with J, the p-p part of J.
trevr_status launch_pp_src(trevr_tree* T, const Scratch& S, uint32_t b0, uint32_t nb,
                           uint32_t cnt, const uint8_t* active, double* J);

}  // namespace trevr
