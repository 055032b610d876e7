// Mean intensity J at active elements on gfx950 (Sections 2.1-2.6 of
// Wadsley, Baumschlager & Shen 2023).
//
// Per active bucket (a leaf of the radiation tree holding >= 1 active
// element) the work is split over kernels:
//   k_active_buckets  list buckets with active members;
//   k_setup           p-p radius by fixed point (wavefront range queries),
//                     p-p set size and number of luminous p-p elements;
//   k_near_fill       the p-p set, luminous elements first;
//   k_walk            one wavefront walks the tree cooperatively (LDS stack,
//                     ballot compaction) and writes the bucket's cut: accepted
//                     cells, opened buckets and resolved element sources, each
//                     source tagged with its HEALPix pixel;
//   k_pp_rays         256 threads per bucket take (p-p element, receiver)
//                     pairs, each testing the rays of the element's HEALPix
//                     ring range: per receiver and ray the p-p optical depth
//                     (kept for the far field);
//   k_pp_src          the attenuated p-p sources (J starts with these):
//                     element-major for sets of 256 or more (or whose pairs
//                     fit one pass), culled by spheres of 16 elements, the
//                     cylinder and the round cone around each source run
//                     before the exact tests; pair-major over culling boxes
//                     otherwise;
//   k_far             256 threads per bucket reduce the cut: sources are
//                     staged per group of 64 rays and sorted along each ray;
//                     every thread takes absorbing cut entries, finds the rays
//                     that cross them and adds the chord's optical depth to
//                     the sources on those rays (LDS atomics); then the
//                     threads sweep the sources against every receiver (FP64
//                     sums), add the background and apply the thick-element
//                     factor.
// Decisions (opening test, p-p membership, the side of a receiver an element
// lies on, pixel of a source, ray-box intersection) are made in FP64 with the
// same correctly rounded operation sequence as their definition, so they are
// reproducible; transcendental physics (exp, the intensity kernel) runs in
// FP32 with FP64 accumulation.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <unordered_map>

#include "path_device.hpp"
#include "path_host.hpp"

namespace trevr {

// ------------------------------------------------------ active buckets
// One row of the grid per scene (blockIdx.y); buckets of all scenes are
// appended to one list, with their scene.
__global__ void k_active_buckets(const DevTree* __restrict__ TT, const uint8_t* active,
                                 uint32_t* blist, uint32_t* bscene, uint32_t* bnact,
                                 uint32_t* nb) {
  const DevTree& T = TT[blockIdx.y];
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= T.num_nodes) return;
  const uint4 nk = T.nk[p];
  if (!(nk.w & META_LEAF)) return;
  const uint8_t* act = active ? active + T.eoff : nullptr;
  const uint2 lk = T.nlink[p];
  uint32_t cnt = 0;
  for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) cnt += (act == nullptr || act[T.perm[s]]) ? 1u : 0u;
  if (cnt == 0) return;
  const uint32_t b = atomicAdd(nb, 1u);
  blist[b] = (uint32_t)p;
  bscene[b] = blockIdx.y;
  bnact[b] = cnt;
}

// Order-independent 64-bit fingerprint of the active set: the sum over
// active input indices i of a 64-bit mix of i (splitmix64 finaliser).  A
// backward call compares it with the forward's to decide whether the
// forward's bucket setup, walks and p-p columns still apply.
__device__ inline unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// A few workgroups per scene, each striding over the elements and adding
// its sum with one atomic (one atomic per wavefront over all elements queued
// thousands of them on the one address).
constexpr unsigned kHashBlocks = 128;
__global__ void __launch_bounds__(256) k_active_hash(const DevTree* __restrict__ TT,
                                                     const uint8_t* active,
                                                     unsigned long long* out) {
  __shared__ unsigned long long part[4];
  const DevTree& T = TT[blockIdx.y];
  unsigned long long v = 0ull;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < T.n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (active == nullptr || active[T.eoff + i]) v += mix64((unsigned long long)(T.eoff + i) + 1ull);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long sum = part[0] + part[1] + part[2] + part[3];
    if (sum) atomicAdd(out, sum);
  }
}

// p-p radius (Section 2.4): past every bucket member by its size, then grown
// until no element inside is wider than the beam there (w r).  One
// wavefront per bucket.
// Each round queries only the shell the sphere grew by.  The shells are
// disjoint and together make up the final sphere, so their elements are the
// p-p set: the rounds leave it as runs (NearOut) in the bucket's stage_cap
// staging words, {run count or kNoRuns, unused, runs...}, for k_near_fill.
// Also records the radius before the last growth (-1 if it never grew) and
// the element whose size set the final radius by that growth (the smallest
// sorted slot among equal sizes), for the adjoint.
template <int SC>
__global__ void __launch_bounds__(64) k_setup(const DevTree* __restrict__ TT, Items I,
                                              const uint32_t* blist, const uint32_t* bscene,
                                              double* brad, double* bprev, uint32_t* barg,
                                              uint32_t* ncnt, uint32_t* nlumc, uint32_t* ovf,
                                              uint32_t* stage, uint32_t stage_cap) {
  __shared__ uint32_t stack[SC];
  const int lane = threadIdx.x;
  const uint32_t b = grid_item(I);
  if (b == kNoItem) return;
  const DevTree& T = TT[bscene[b]];
  const uint32_t leaf = blist[b];
  double c[3];
  leaf_centre(T, leaf, c);
  double r = 0.0, rprev = -1.0;
  uint32_t cnt = 0, nlum = 0, arg = 0xFFFFFFFFu;
  bool overflow = false;
  NearOut o{stage_cap ? stage + (size_t)b * stage_cap + 2 : nullptr, true, 0u, 0u, 0u,
            stage_cap ? (stage_cap - 2u) / 2u : 0u};
  if (T.flags & TREVR_NEAR_FIELD) {
    r = T.rpp_min;
    const uint2 lk = T.nlink[leaf];
    double rm = 0.0;
    for (uint32_t s = lk.x + lane; s < lk.x + lk.y; s += 64)
      rm = fmax(rm, sqrt(dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c)) + T.h[s]);
    r = fmax(r, wave_max(rm));
    // each round counts only the shell the sphere grew by; the widest
    // element so far (smallest slot among equal sizes) is kept across rounds
    double r2in = -1.0, hw = 0.0;
    uint32_t hwa = 0xFFFFFFFFu;
    for (;;) {
      double hm = 0.0;
      uint32_t ha = 0xFFFFFFFFu, nl = 0;
      cnt += wave_near(T, c, r * r, stack, stack_cap<SC>(T), &hm, &nl, o, &overflow, &ha, r2in);
      nlum += nl;
      if (hm > hw || (hm == hw && ha < hwa)) {
        hw = hm;
        hwa = ha;
      }
      const double rn = fmax(r, hw / T.wbeam);
      if (!(rn > r) || overflow) break;
      r2in = r * r;
      rprev = r;
      r = rn;
      arg = hwa;   // the widest element inside the sphere set the new radius
    }
  }
  if (lane == 0) {
    brad[b] = r;
    bprev[b] = rprev;
    barg[b] = arg;
    ncnt[b] = cnt;
    nlumc[b] = nlum;
    if (stage_cap) stage[(size_t)b * stage_cap] = o.out ? o.nrun : kNoRuns;
    if (overflow) atomicOr(ovf, OVF_SETUP);
  }
}

// One workgroup (one wavefront) per bucket: a plain grid, since most buckets
// take a few microseconds, too short to be worth a work-queue claim.  A
// bucket whose set k_setup staged writes it in slot order, which keeps
// consecutive list entries close in space for the p-p kernels' culling
// boxes: its runs are sorted in LDS by (first slot, staging index) (bitonic,
// the staging index breaks ties between two shells' members of one window),
// then placed by a prefix over their member counts.  The others query the
// sphere again (the same sphere as the last query of k_setup, so the same
// stack suffices) and, for trees of up to 64 x (LDS words) elements, are put
// in slot order through a bitmap.
template <int SC>
__global__ void __launch_bounds__(64) k_near_fill(const DevTree* __restrict__ TT,
                                                  const uint32_t* rng, const uint32_t* blist,
                                                  const uint32_t* bscene, const double* brad,
                                                  const uint32_t* noff, const uint32_t* nlumc,
                                                  const uint32_t* bsrc,
                                                  const uint32_t* __restrict__ stage,
                                                  uint32_t stage_cap,
                                                  uint32_t* __restrict__ nidx) {
  constexpr int kWords = SC / 2 > (int)kSortRuns ? SC / 2 : (int)kSortRuns;
  __shared__ unsigned long long lds[kWords];   // the traversal stack, or sort keys
  const uint32_t lane = threadIdx.x;
  const uint32_t b = blockIdx.x;
  if (b >= rng[1]) return;
  const DevTree& T = TT[bscene[b]];
  if (!(T.flags & TREVR_NEAR_FIELD)) return;
  const uint32_t nl = nlumc[b];
  uint32_t* out = nidx + noff[b];
  const uint32_t* sg = stage_cap ? stage + (size_t)bsrc[b] * stage_cap : nullptr;
  const uint32_t nrun = sg ? sg[0] : kNoRuns;
  if (nrun != kNoRuns) {
    const uint2* run = reinterpret_cast<const uint2*>(sg + 2);
    uint32_t P = 2;
    while (P < nrun) P <<= 1;
    for (uint32_t t = lane; t < P; t += 64)
      lds[t] = t < nrun ? ((unsigned long long)run[t].x << kSortIdxBits) | t : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t q = lane; q < P / 2; q += 64) {
          const uint32_t t = ((q & ~(j - 1u)) << 1) | (q & (j - 1u)), u = t | j;
          const unsigned long long x = lds[t], y = lds[u];
          if ((x > y) == ((t & k) == 0u)) {
            lds[t] = y;
            lds[u] = x;
          }
        }
        __syncthreads();
      }
    }
    uint32_t bl = 0, bd = 0;   // luminous and other members placed so far
    for (uint32_t p0 = 0; p0 < nrun; p0 += 64) {
      const uint32_t p = p0 + lane;
      uint32_t first = 0, m = 0;
      if (p < nrun) {
        const unsigned long long key = lds[p];
        first = (uint32_t)(key >> kSortIdxBits);
        m = run[(uint32_t)key & ((1u << kSortIdxBits) - 1u)].y;
      }
      uint32_t tl, td;
      uint32_t a = bl + wave_excl_bits<kLeafBatchBits>((uint32_t)__popc(m & 0xFFFFu), &tl);
      uint32_t d = nl + bd + wave_excl_bits<kLeafBatchBits>((uint32_t)__popc(m >> 16), &td);
#pragma unroll
      for (int k = 0; k < kLeafBatch; ++k) {
        if ((m >> k) & 1u) out[a++] = first + (uint32_t)k;
        if ((m >> (16 + k)) & 1u) out[d++] = first + (uint32_t)k;
      }
      bl += tl;
      bd += td;
    }
    return;
  }
  double c[3];
  leaf_centre(T, blist[b], c);
  const double r = brad[b];
  bool overflow = false;
  NearOut o{out, false, 0u, nl, 0u, 0u};
  wave_near(T, c, r * r, reinterpret_cast<uint32_t*>(lds), stack_cap<SC>(T), nullptr, nullptr, o,
            &overflow);
  // the queried list into slot order as well, when a bitmap of the tree's
  // slots fits the LDS: each part (luminous, others) marked, then read back
  // in order, a contiguous range of bitmap words per lane
  uint32_t* bits = reinterpret_cast<uint32_t*>(lds);
  constexpr uint32_t kBitWords = 2u * (uint32_t)kWords;
  const uint32_t words = (uint32_t)((T.n + 31) / 32), n = noff[b + 1] - noff[b];
  if (overflow || words > kBitWords) return;
  for (int part = 0; part < 2; ++part) {
    const uint32_t lo = part ? nl : 0u, hi = part ? n : nl;
    if (hi - lo < 2u) continue;
    __syncthreads();
    for (uint32_t w = lane; w < words; w += 64) bits[w] = 0u;
    __syncthreads();
    for (uint32_t k = lo + lane; k < hi; k += 64) {
      const uint32_t e = out[k];
      if (e < (uint32_t)T.n) atomicOr(&bits[e >> 5], 1u << (e & 31u));
    }
    __syncthreads();
    const uint32_t per = (words + 63u) / 64u;
    const uint32_t w0 = min(words, lane * per), w1 = min(words, w0 + per);
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; ++w) cnt += (uint32_t)__popc(bits[w]);
    uint32_t pos = lo + wave_excl(cnt, (int)lane);
    for (uint32_t w = w0; w < w1; ++w) {
      uint32_t m = bits[w];
      while (m && pos < hi) {
        out[pos++] = w * 32u + (uint32_t)(__ffs(m) - 1);
        m &= m - 1u;
      }
    }
  }
}

// ------------------------------------------------------------- the walk
// Cut lists hold cap entries per bucket; a bucket that needs more still
// counts them all (bstat, and the batch maximum in ovf[1]) so the host can
// walk it again with room for them.
template <int SC>
__global__ void __launch_bounds__(64) k_walk(const DevTree* __restrict__ TT, Items I,
                                             const uint32_t* blist, const uint32_t* bscene,
                                             const double* brad, uint2* cut, uint32_t cap,
                                             uint32_t* bstat, uint32_t* ovf) {
  __shared__ uint32_t stack[SC];
  __shared__ uint32_t lfirst[64], lbeg[64];
  const int lane = threadIdx.x;
  const uint32_t bucket = grid_item(I);
  if (bucket == kNoItem) return;
  const DevTree& T = TT[bscene[bucket]];
  const uint32_t leafb = blist[bucket];
  const double r = brad[bucket];
  const double r2 = r * r;
  double c[3];
  leaf_centre(T, leafb, c);
  uint2* out = cut + (size_t)(bucket - I.lo) * cap;
  uint32_t ncut = 0, nsrc = 0, ncells = 0;
  bool overflow = false;
  int sp = 1, maxsp = 1;
  if (lane == 0) stack[0] = 0u;
  __syncthreads();
  while (sp > 0) {
    const int take = min(sp, 64);
    sp -= take;
    const bool valid = lane < take;
    const uint32_t node = valid ? stack[sp + lane] : 0u;
    __syncthreads();
    bool push = false, emit = false, opened = false, isleaf = false;
    uint4 nk = make_uint4(0, 0, 0, 0);
    double4 cn = make_double4(0, 0, 0, 0);
    uint2 nl = make_uint2(0u, 0u);   // loaded with the key, off the tests' path
    if (valid) {
      nk = T.nk[node];
      cn = T.cen[node];
      nl = T.nlink[node];
      double lo[3], hi[3];
      node_box(T.hdr, nk, lo, hi);
      if (!(far2_box(lo, hi, c) < r2)) {
        const double cc[3] = {cn.x, cn.y, cn.z};
        opened = open_cell(lo, hi, cc, c, r2, T.theta2);
        isleaf = (nk.w & META_LEAF) != 0u;
        push = opened && !isleaf;
        emit = !push;
      }
    }
    const uint64_t pm = ballot64(push);
    const int ppos = mbcnt(pm);
    const int npush = __popcll(pm);
    if (sp + 2 * npush > stack_cap<SC>(T)) {
      overflow = true;
      break;
    }
    if (push) {
      stack[sp + 2 * ppos] = nl.x;                 // child 1
      stack[sp + 2 * ppos + 1] = node + 1u;        // child 0
    }
    sp += 2 * npush;
    maxsp = max(maxsp, sp);
    ncells += (uint32_t)__popcll(ballot64(emit));
    // cell entries: absorbers and merged sources
    uint32_t meta = 0u;
    bool write = false;
    if (emit) {
      const bool absorbing = (nk.w & META_ABS) != 0u;
      if (opened) {  // opened bucket: its absorption, sources resolved below
        meta = CUT_LEAF | CUT_NOPIX | (absorbing ? CUT_ABS : 0u);
        write = absorbing;
      } else {
        uint32_t pix = CUT_NOPIX;
        if (nk.w & META_LUM) pix = source_pixel(T.nside, cn.x - c[0], cn.y - c[1], cn.z - c[2]);
        meta = CUT_CELL | pix | (absorbing ? CUT_ABS : 0u);
        write = absorbing || (pix != CUT_NOPIX);
      }
    }
    const uint64_t wm = ballot64(write);
    if (write) {
      const uint32_t idx = ncut + (uint32_t)mbcnt(wm);
      if (idx < cap) out[idx] = make_uint2(node, meta);
    }
    ncut += (uint32_t)__popcll(wm);
    nsrc += (uint32_t)__popcll(ballot64(write && ((meta & 0xFFFFu) != CUT_NOPIX)));
    // element sources of opened luminous buckets, outside the p-p sphere:
    // the (bucket, element) pairs of this step spread over the lanes, in
    // lane order then element order
    const bool lumleaf = emit && opened && (nk.w & META_LUM);
    const uint2 llk = lumleaf ? nl : make_uint2(0u, 0u);
    const uint32_t lbase = wave_excl(llk.y, lane);
    const uint32_t ltot = (uint32_t)__shfl((int)(lbase + llk.y), 63);
    if (ltot) {
      lfirst[lane] = llk.x;
      lbeg[lane] = lbase;
      __syncthreads();
      for (uint32_t e0 = 0; e0 < ltot; e0 += 64) {
        const uint32_t e = e0 + (uint32_t)lane;
        bool is_src = false;
        uint32_t pix = 0u, s = 0u;
        if (e < ltot) {
          int lo = 0, hi = 63;   // the last lane whose elements start at or before e
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lbeg[mid] <= e) lo = mid; else hi = mid - 1;
          }
          s = lfirst[lo] + (e - lbeg[lo]);
          const double lb = T.lbol[s];
          const double px = (double)T.x[s], py = (double)T.y[s], pz = (double)T.z[s];
          if (lb > 0.0 && !(dist2_pt3(px, py, pz, c) < r2)) {
            is_src = true;
            pix = source_pixel(T.nside, px - c[0], py - c[1], pz - c[2]);
          }
        }
        const uint64_t sm = ballot64(is_src);
        if (is_src) {
          const uint32_t idx = ncut + (uint32_t)mbcnt(sm);
          if (idx < cap) out[idx] = make_uint2(s, CUT_PART | pix);
        }
        ncut += (uint32_t)__popcll(sm);
        nsrc += (uint32_t)__popcll(sm);
      }
    }
    __syncthreads();
  }
  if (lane == 0) {
    bstat[4 * bucket + 0] = ncut;
    bstat[4 * bucket + 1] = nsrc;
    bstat[4 * bucket + 2] = ncells;
    if (overflow) atomicOr(ovf, OVF_WALK);
    if (ncut > __atomic_load_n(ovf + 1, __ATOMIC_RELAXED)) atomicMax(ovf + 1, ncut);
    atomic_max_u64(&T.counters[CNT_MAX_CUT], ncut);
    atomic_max_u64(&T.counters[CNT_MAX_STACK], (unsigned long long)maxsp);
  }
}

// For each receiver i and ray k: the optical depth of the p-p elements ahead
// of i on the ray (exact FP64 projection: a discontinuous decision) whose
// size h reaches the ray line (b < h, with b^2 = |d|^2 - proj^2: continuous,
// Sigma -> 0 at b = h): kappa_l Sigma_l(b), Sigma_l(b) = 3 m_l/(pi h_l^2)
// (1 - b/h_l).  Written to tpp[receiver][ray][band] for the far field.
//
// Element-major: per receiver chunk and group of rays (all of them up to
// N_side 4 and four bands, else 64), threads take (p-p element, receiver)
// pairs; a pair tests only the group's rays in the element's ring range (and
// the directed ray), 64 at a time first with a conservative FP32 test, then
// with the exact FP64 one, and adds each hit's kappa Sigma to the (receiver,
// ray) sums in LDS, written out once per group.
template <int NB>
__global__ void __launch_bounds__(kNT) k_pp_rays(const DevTree* __restrict__ TT, Items I,
                                                const uint32_t* blist, const uint32_t* bscene,
                                                const uint32_t* noff, const uint32_t* nidx,
                                                const uint32_t* toff, const uint8_t* active,
                                                float* tpp) {
  constexpr int RGN = PpRayGroup<NB>::value;
  const int t = threadIdx.x;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, s_item;
  __shared__ double rn[RGN][3];
  __shared__ float rnf[RGN][3];
  __shared__ float acc[kRMax][RGN][NB];
  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0;
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  const int64_t n = T.n;
  float* tppb = tpp + toff[bucket];
  double ud[3];
  const int kd = directed_ray(T, c, ud);   // the bucket's directed ray, if any
  uint32_t ract = 0;
  uint32_t member = lk.x;
  for (;;) {
    const int nrecv = load_receivers(T, act, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    for (int k0 = 0; k0 < nray; k0 += RGN) {
      const int kn = min(RGN, nray - k0);
      // the directed ray, when it is in this group: its direction is not a
      // HEALPix centre, so it is tested whatever the ring range
      const int kdg = (kd >= k0 && kd < k0 + kn) ? kd - k0 : -1;
      if (t < kn) {
        const int k = k0 + t;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double na = (k == kd) ? ud[a] : T.ray_n[3 * k + a];
          rn[t][a] = na;
          rnf[t][a] = (float)na;
        }
      }
      for (int q = t; q < kRMax * RGN * NB; q += kNT) (&acc[0][0][0])[q] = 0.0f;
      __syncthreads();
      for (uint32_t pq = (uint32_t)t; pq < nnear * (uint32_t)nrecv; pq += kNT) {
        const uint32_t u = pq / (uint32_t)nrecv;
        const int i = (int)(pq % (uint32_t)nrecv);
        const uint32_t l = near[u];
        if (l == recv[i].slot) continue;
        const double d0 = (double)T.x[l] - recv[i].x[0];
        const double d1 = (double)T.y[l] - recv[i].x[1];
        const double d2 = (double)T.z[l] - recv[i].x[2];
        const double dd = d0 * d0 + d1 * d1 + d2 * d2;
        const double hl = T.h[l];
        const double h2 = hl * hl;
        const float df[3] = {(float)d0, (float)d1, (float)d2};
        const float ddf = (float)dd;
        const float lim = (float)(dd - h2) - 1e-5f * ddf - 1e-30f;
        const float neg = -1e-5f * cull_sqrt(ddf);
        int ka, kb;
        ray_ring_range(T.nside, d0, d1, d2, dd, h2, &ka, &kb);
        const int lo = max(ka - k0, 0), hi = min(kb - k0, kn);
        bool loaded = false;
        float sig = 0.0f, iv = 0.0f, kap[NB];
        // candidates 64 rays at a time: the FP32 test, then the exact one
        for (int s0 = 0; s0 < kn; s0 += 64) {
          uint64_t cand = 0ull;
          for (int kq = max(lo, s0); kq < min(hi, s0 + 64); ++kq) {
#pragma clang fp contract(fast)   // FP32 test with margins: fused products are fine
            const float pf = rnf[kq][0] * df[0] + rnf[kq][1] * df[1] + rnf[kq][2] * df[2];
            if (pf > neg && pf * pf >= lim) cand |= 1ull << (kq - s0);
          }
          if (kdg >= s0 && kdg < s0 + 64) {
            const float pf = rnf[kdg][0] * df[0] + rnf[kdg][1] * df[1] + rnf[kdg][2] * df[2];
            if (pf > neg && pf * pf >= lim) cand |= 1ull << (kdg - s0);
          }
          if (cand == 0ull) continue;
          if (!loaded) {
            // column density scale 3m/(pi h^2) and 1/h in FP32 (values,
            // not decisions; no FP64 divisions in this VALU-bound loop)
            iv = __builtin_amdgcn_rcpf((float)hl);
            sig = (float)(3.0 / kPi) * T.m[l] * iv * iv;
#pragma unroll
            for (int b = 0; b < NB; ++b) kap[b] = T.kappa[(int64_t)b * n + l];
            loaded = true;
          }
          while (cand) {
            const int kq = s0 + __ffsll((long long)cand) - 1;
            cand &= cand - 1ull;
            const double proj = d0 * rn[kq][0] + d1 * rn[kq][1] + d2 * rn[kq][2];
            const double b2 = dd - proj * proj;
            if (!(proj > 0.0 && b2 < h2)) continue;
            const float bb = __builtin_amdgcn_sqrtf((float)fmax(b2, 0.0));
            const float sg = sig * (1.0f - bb * iv);
#pragma unroll
            for (int b = 0; b < NB; ++b) atomicAdd(&acc[i][kq][b], kap[b] * sg);
          }
        }
      }
      __syncthreads();
      for (int q = t; q < nrecv * kn; q += kNT) {
        const int i = q / kn, kq = q % kn;
        float* o = tppb + ((int64_t)(ract + i) * nray + k0 + kq) * NB;
#pragma unroll
        for (int b = 0; b < NB; ++b) o[b] = acc[i][kq][b];
      }
      __syncthreads();
    }
    ract += (uint32_t)nrecv;
  }
  }
}

// Adds (none when dst is null) and clears the p-p source kernel's counter
// sums: near pairs, (receiver, source, element) triples, the largest set,
// the triples whose element absorbs on the path and the job-log entries.
__device__ inline void pp_counters_flush(unsigned long long* dst, unsigned long long* s) {
  if (dst) {
    if (s[0]) atomicAdd(&dst[CNT_NEAR_PAIRS], s[0]);
    if (s[1]) atomicAdd(&dst[CNT_NS_TRIPLES], s[1]);
    if (s[2]) atomic_max_u64(&dst[CNT_MAX_NEAR], s[2]);
    if (s[3]) atomicAdd(&dst[CNT_NS_HITS], s[3]);
    if (s[4]) atomicAdd(&dst[CNT_PP_LOG], s[4]);
  }
  s[0] = s[1] = s[2] = s[3] = s[4] = 0ull;
}

// For each receiver i and luminous p-p element j (i itself included, at
// r = 0): L_j K(r_ij, h_i) exp(-tau_ij), tau over the p-p elements closer to
// j than i is (exact FP64 squared distances: discontinuous) and within their
// size of the segment i-j (continuous).  J of i starts with the sum.
//
// The optical depth of each pair is kept in ptau [pair][band] (pairs of a
// bucket from poff[bucket], receiver-chunk-major, then (source, receiver)),
// for the adjoint.  J == nullptr: only ptau is written.
template <int NB>
__global__ void __launch_bounds__(kNT, 4) k_pp_src(const DevTree* __restrict__ TT, Items I,
                                               const uint32_t* blist, const uint32_t* bscene,
                                               const uint32_t* noff, const uint32_t* nlumc,
                                               const uint32_t* nidx, const uint32_t* poff,
                                               const uint8_t* active, double* Jall,
                                               float* ptau, int sub, JobLog JL) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // the staged elements (pair-major passes), the exact-test job queues
  // (element-major passes) and the receiver sums share their LDS
  __shared__ union {
    NearTile<NB> S;
    struct {
      uint16_t qa[kNT / 64][kJobQ];   // per-element test passes (lane, run)
      uint32_t xl[kNT / 64][kJobQ];   // round-cone passes: element ...
      uint8_t xq[kNT / 64][kJobQ];    // ... and run, for the exact tests
      // per lane of a wavefront: its element relative to the bucket centre
      // with its size, and its slot, read by the lanes that test it (one
      // LDS read instead of four shuffles: 542 -> 528 ms on the batched
      // workload)
      float4 ep[kNT / 64][64];
      uint32_t el[kNT / 64][64];
    } JQ;
    double red[kNT][NB];
  } U;
  NearTile<NB>& S = U.S;
  double (*red)[NB] = U.red;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, s_item;
  // each thread's pair, for lanes that test it on the thread's behalf; the
  // optical depths gathered for it by other lanes (tacc)
  __shared__ float pd_xj[kNT][3];   // FP32 as stored, widened where read
  __shared__ double pd_r2[kNT], pd_inv2[kNT];
  __shared__ uint32_t pd_j[kNT];
  __shared__ float pd_jr[kNT][3], pd_jinv[kNT], pd_jlim[kNT], pd_k2[kNT], pd_m2[kNT];
  __shared__ float tacc[kNT][NB];
  __shared__ uint8_t nlist[kNT / 64][64];
  __shared__ float egrp[kNT / 64][4][5];   // per wavefront: element spheres of its quarters
  // the workgroup's sums of the per-bucket counters (thread 0), added to a
  // scene's counters when it turns to another scene and after its last bucket
  __shared__ unsigned long long csum[5];   // near pairs, triples, largest set, hits, log
  __shared__ unsigned long long* cdst;
  __shared__ unsigned long long s_hits;    // this bucket's hits so far
  __shared__ unsigned long long s_logn;    // this bucket's job-log entries so far
  __shared__ uint32_t s_logbad;            // the log does not cover this bucket
  if (threadIdx.x == 0) {
    cdst = nullptr;
    csum[0] = csum[1] = csum[2] = csum[3] = csum[4] = 0ull;
    s_hits = 0ull;
    s_logn = 0ull;
  }
  uint32_t hits = 0;   // this thread's exact-test passes in the current bucket
  uint32_t logn = 0;   // the wavefront's job-log entries in the current bucket
  LogPos lp{kLogFresh, 0u};   // the wavefront's job-log stream
  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  double* J = Jall ? Jall + T.joff : nullptr;
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0, nl = nlumc[bucket];
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int64_t n = T.n;
  uint32_t member = lk.x;
  uint32_t nact = 0;
  LogPos lbeg{kLogNone, 0u};   // where this bucket's stream starts
  if (t == 0) s_logbad = 0u;
  for (;;) {
    const int nrecv = load_receivers(T, act, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    float* pt = ptau + (int64_t)poff[bucket] + (int64_t)nact * nl * NB;
    nact += (uint32_t)nrecv;
    const int stride = (kNT / nrecv) * nrecv;       // thread t keeps receiver t % nrecv
    const int i = t % nrecv;
    const RecvInfo& ri = recv[i];
    const double xi0 = ri.x[0], xi1 = ri.x[1], xi2 = ri.x[2];
    const uint32_t si = ri.slot;
    const bool em = nnear >= kPpElementMajor || (uint32_t)nrecv * nl <= (uint32_t)kNT;
    if (JL.log) {
      if ((!em || nnear >= kLogMaxNear) && t == 0) s_logbad = 1u;
      if (em && lbeg.blk == kLogNone && log_ready(JL, lp)) lbeg = lp;
    }
    float reach = 0.0f;   // largest receiver distance from the centre
    for (int k = 0; k < nrecv; ++k)
      reach = fmaxf(reach, sqrtf(recv[k].rel[0] * recv[k].rel[0] + recv[k].rel[1] * recv[k].rel[1] +
                                 recv[k].rel[2] * recv[k].rel[2]));
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    const uint32_t P = (uint32_t)nrecv * nl;
    for (uint32_t pb = 0; pb < P; pb += (uint32_t)stride) {
      const uint32_t p = pb + (uint32_t)t;
      const bool ok = t < stride && p < P;
      const uint32_t j = ok ? near[p / nrecv] : near[0];
      const double xj0 = (double)T.x[j], xj1 = (double)T.y[j], xj2 = (double)T.z[j];
      const double e0 = xj0 - xi0, e1 = xj1 - xi1, e2 = xj2 - xi2;
      const double rij2 = e0 * e0 + e1 * e1 + e2 * e2;
      const double inv2 = rij2 > 0.0 ? 1.0 / rij2 : 0.0;
      const float jr[3] = {(float)(xj0 - c[0]), (float)(xj1 - c[1]), (float)(xj2 - c[2])};
      float smin[3], smax[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        smin[a] = fminf(ri.rel[a], jr[a]);
        smax[a] = fmaxf(ri.rel[a], jr[a]);
      }
      const float r2f = (float)rij2 * (1.0f + 1e-5f) + 1e-30f;
      // the segment i -> j for the FP32 culling (relative to the bucket centre)
      const float sd[3] = {jr[0] - ri.rel[0], jr[1] - ri.rel[1], jr[2] - ri.rel[2]};
      float sinv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) sinv[a] = (sd[a] != 0.0f) ? 1.0f / sd[a] : 0.0f;
      float tau[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        tau[b] = 0.0f;
        tacc[t][b] = 0.0f;
      }
      pd_xj[t][0] = (float)xj0;   // exact: the positions are FP32
      pd_xj[t][1] = (float)xj1;
      pd_xj[t][2] = (float)xj2;
      // a pair without a path (past the pairs, or the receiver itself) gets
      // a negative squared length, which fails the exact test
      pd_r2[t] = (ok && rij2 > 0.0) ? rij2 : -1.0;
      pd_inv2[t] = inv2;
      pd_j[t] = j;
      if (em) {
        // ---- element-major: each lane owns a p-p element; per source run
        // (the nrecv pairs of one source) it tests the element against the
        // cylinder of the receivers' reach around the centre's segment to
        // the source, and the element no farther from the source than the
        // farthest receiver; passing (element, source run) jobs are queued
        // per wavefront, filtered 64 at a time by the round cone (the
        // reach at the centre, none at the source), and run 64 at a time
        // with the exact FP64 test of the pair-major sweep on each pair of
        // the run, LDS atomics adding into tacc.  Both tests are supersets
        // of the exact test's passes
        run_tab_entry(jr, reach, pd_jr, pd_jinv, pd_jlim, pd_k2, pd_m2, t);
        const RunTab RT{pd_jr, pd_jinv, pd_jlim, pd_k2, pd_m2};
        const float Rm = reach * (1.0f + 1e-5f);
        __syncthreads();
        const int qend = (int)min((uint32_t)stride, P - pb);   // pairs of this pass
        uint16_t* QA = U.JQ.qa[wv];
        uint32_t* XL = U.JQ.xl[wv];
        uint8_t* XQ = U.JQ.xq[wv];
        uint32_t head = 0, tail = 0;   // the exact-test queue, kept across chunks
        // the job log: this pass's number of records (written at its end),
        // then per chunk with jobs a record and the jobs as they pass the
        // round cone
        const size_t lpass = JL.log ? log_put(JL, lp, 1u, lane == 0, 0u, 0) : ~(size_t)0;
        uint32_t nrec = 0, cnext = 0;
        // one batch of up to 64 queued exact-test jobs, job head + lane on
        // this lane: a job is (element, source run); its lane reads the
        // element and runs the exact test on each of the run's nrecv pairs
        // (pair q0 + k has receiver k), the source read once
        auto run_jobs = [&](uint32_t cnt) {
          if ((uint32_t)lane < cnt) {
            const uint32_t slot = (head + (uint32_t)lane) & (kJobQ - 1);
            const uint32_t vl = XL[slot];
            const int q0 = XQ[slot];
            const double vx = (double)T.x[vl], vy = (double)T.y[vl], vz = (double)T.z[vl];
            const double vhl = T.h[vl];
            const double vh2 = vhl * vhl;
            // column density scale 3m/(pi h^2) and 1/h in FP32 (they set the
            // values added, not the decisions)
            const float viv = __builtin_amdgcn_rcpf((float)vhl);
            const float vsig = (float)(3.0 / kPi) * T.m[vl] * viv * viv;
            float vkap[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) vkap[b] = T.kappa[(int64_t)b * n + vl];
            const double qx0 = (double)pd_xj[q0][0], qx1 = (double)pd_xj[q0][1],
                         qx2 = (double)pd_xj[q0][2];
            const uint32_t qj = pd_j[q0];
            const double f0 = vx - qx0, f1 = vy - qx1, f2 = vz - qx2;
            const double ff = f0 * f0 + f1 * f1 + f2 * f2;
            // four receivers per step, every condition evaluated: their LDS
            // reads issue together instead of one wait per condition
            // (forward p-p sources 582 -> 568 ms at two per step on the
            // batched workload, 512 -> 505 ms from two to four; unrolled
            // fully, the spills cost more than the waits)
#pragma unroll 4
            for (int k = 0; k < nrecv; ++k) {
              const int q = q0 + k;
              const RecvInfo& rq = recv[k];
              const double pe0 = qx0 - rq.x[0], pe1 = qx1 - rq.x[1], pe2 = qx2 - rq.x[2];
              const double w0 = vx - rq.x[0], w1 = vy - rq.x[1], w2 = vz - rq.x[2];
              double uu = (w0 * pe0 + w1 * pe1 + w2 * pe2) * pd_inv2[q];
              uu = fmin(1.0, fmax(0.0, uu));
              const double g0 = w0 - uu * pe0, g1 = w1 - uu * pe1, g2 = w2 - uu * pe2;
              const double b2 = g0 * g0 + g1 * g1 + g2 * g2;
              if ((ff < pd_r2[q]) & (b2 < vh2) & (vl != rq.slot) &
                  (vl != qj)) {
                ++hits;
                // the hardware square root (about an ulp): it sets the value
                // added, not the decision (batched forward 8 ms, adjoint 12 ms
                // less than the correctly rounded one)
                const float bb = __builtin_amdgcn_sqrtf((float)b2);
                const float sg = vsig * (1.0f - bb * viv);
#pragma unroll
                for (int b = 0; b < NB; ++b) atomicAdd(&tacc[q][b], vkap[b] * sg);
              }
            }
          }
        };
        for (uint32_t c0 = 0; c0 < nnear; c0 += kNT) {
          const uint32_t u = c0 + (uint32_t)t;
          const bool has = u < nnear;
          const uint32_t l = has ? near[u] : near[0];
          // the lane keeps what the element tests need; an exact-test job
          // reads the rest of its element itself
          const double hl = T.h[l];
          const float pr[3] = {(float)((double)T.x[l] - c[0]), (float)((double)T.y[l] - c[1]),
                               (float)((double)T.z[l] - c[2])};
          // no element: a NaN size, which fails every element test (one
          // read less per test: forward p-p sources 562 -> 541 ms with the
          // quarter pair selected without branches)
          const float hrad = has ? (float)hl * (1.0f + 1e-5f) +
                                       1e-5f * (fabsf(pr[0]) + fabsf(pr[1]) + fabsf(pr[2]))
                                 : __int_as_float(0x7fc00000);
          U.JQ.ep[wv][lane] = make_float4(pr[0], pr[1], pr[2], hrad);
          U.JQ.el[wv][lane] = l;
          wave_lds_sync();
          uint32_t ha = 0, ta = 0;   // wave-uniform cursors of the first queue
          uint32_t lcnt = 0;             // this chunk's jobs
          size_t lrec = ~(size_t)0;      // its record
          // the round-cone filter over up to 64 jobs of the first queue (job
          // ha + lane on this lane); the survivors go to the exact tests
          auto filter_jobs = [&](uint32_t cnt) {
            const bool mine = (uint32_t)lane < cnt;
            const uint16_t job = QA[(ha + (uint32_t)lane) & (kJobQ - 1)];
            const int L = mine ? (int)(job >> 8) : lane;
            const float4 e4 = U.JQ.ep[wv][L];
            const float vp[3] = {e4.x, e4.y, e4.z};
            const float vh = e4.w;
            const uint32_t vl = U.JQ.el[wv][L];
            const int q0 = (int)(job & 0xFFu);
            const bool keep = mine && elem_run_cone(vp, vh, RT, Rm, q0);
            const uint64_t m = ballot64(keep);
            if (keep) {
              const uint32_t slot = (tail + (uint32_t)mbcnt(m)) & (kJobQ - 1);
              XL[slot] = vl;
              XQ[slot] = (uint8_t)q0;
            }
            tail += (uint32_t)__popcll(m);
            if (JL.log && m != 0ull) {
              if (lcnt == 0u) lrec = log_record(JL, lp);
              log_put(JL, lp, (uint32_t)__popcll(m), keep, (uint32_t)mbcnt(m), job);
            }
            lcnt += (uint32_t)__popcll(m);
            wave_lds_sync();
            while (tail - head >= 64u) {
              run_jobs(64u);
              head += 64u;
            }
          };
          // the wavefront's elements as one sphere first: only the source
          // runs that may reach it go through the per-element tests
          elem_group(pr, hrad, has, egrp[wv]);
          const int nruns = qend / nrecv;
          for (int k0 = 0; k0 < nruns; k0 += kElemGroup) {
            uint64_t gm = group_runs(egrp[wv], RT, Rm, k0, nruns, nrecv);
            while (gm != 0ull) {
              // four (quarter, run) pairs at a time, 16 lanes each: lane
              // 16 i + j tests element j of its pair's quarter
              const int pq = take_quarter_pair(&gm);
              const int eL = pq >= 0 ? (pq >> 4) * kElemGroup + (lane & (kElemGroup - 1)) : lane;
              const int q0 = pq >= 0 ? (k0 + (pq & (kElemGroup - 1))) * nrecv : 0;
              const float4 e4 = U.JQ.ep[wv][eL];
              const float vp[3] = {e4.x, e4.y, e4.z};
              const float vh = e4.w;
              const bool pass = (pq >= 0) & elem_run_test(vp, vh, RT, Rm, q0);
              const uint64_t m = ballot64(pass);
              if (m == 0ull) continue;
              if (pass) QA[(ta + (uint32_t)mbcnt(m)) & (kJobQ - 1)] = (uint16_t)((eL << 8) | q0);
              ta += (uint32_t)__popcll(m);
              wave_lds_sync();
              while (ta - ha >= 64u) {
                filter_jobs(64u);
                ha += 64u;
              }
            }
          }
          if (ta > ha) filter_jobs(ta - ha);
          if (lcnt != 0u) {
            const uint32_t cc = c0 / (uint32_t)kNT;
            if (lrec != ~(size_t)0 && lane == 0) {
              JL.log[lrec] = (uint16_t)(cc - cnext);
              JL.log[lrec + 1] = (uint16_t)lcnt;
            }
            cnext = cc + 1u;
            ++nrec;
            logn += 3u + lcnt;   // the record, a block end it may skip, the jobs
          }
          wave_lds_sync();
        }
        if (tail > head) run_jobs(tail - head);
        if (lpass != ~(size_t)0 && lane == 0) JL.log[lpass] = (uint16_t)nrec;
        logn += 1u;
        wave_lds_sync();
        __syncthreads();
      } else
      for (uint32_t c0 = 0; c0 < nnear; c0 += kNChunk) {
        const uint32_t cl = min((uint32_t)kNChunk, nnear - c0);
        stage_near<NB>(S, T, near, c0, cl, c);
        const int nsub = ((int)cl + sub - 1) / sub;
        const float (*BL)[3] = near_boxes(S, sub, false);
        const float (*BH)[3] = near_boxes(S, sub, true);
        for (int sb = 0; sb < nsub; ++sb) {
          bool need = false;
          if (ok && rij2 > 0.0) {
            // the sub-box (elements grown by their size) must meet the
            // segment, and come nearer to j than i is
            float dmin2 = 0.0f, t0 = 0.0f, t1 = 1.0f;
            bool over = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const float lo = BL[sb][a], hi = BH[sb][a];
              over = over && (smax[a] >= lo) && (smin[a] <= hi);
              if (sd[a] != 0.0f) {
                const float u = (lo - ri.rel[a]) * sinv[a], v = (hi - ri.rel[a]) * sinv[a];
                t0 = fmaxf(t0, fminf(u, v));
                t1 = fminf(t1, fmaxf(u, v));
              }
              const float dj = fmaxf(fmaxf(lo - jr[a], jr[a] - hi), 0.0f);
              dmin2 += dj * dj;
            }
            need = over && t0 <= t1 + 1e-4f && dmin2 < r2f;
          }
          const uint64_t m = ballot64(need);
          if (m == 0ull) continue;
          const int nneed = __popcll(m);
          const int per = 64 / sub;   // lanes served per round when spread
          const int u1 = min((int)cl, (sb + 1) * sub);
          if (2 * ((nneed + per - 1) / per) < sub) {
            // few lanes need this sub-box: their (pair, element) tests spread
            // over the wavefront, sub lanes (one element each) per pair, the
            // same FP64 operation sequence as below
            if (need) nlist[wv][mbcnt(m)] = (uint8_t)lane;
            wave_lds_sync();
            const int grp = lane / sub, u = sb * sub + (lane - grp * sub);
            for (int r0 = 0; r0 < nneed; r0 += per) {
              const int which = r0 + grp;
              const bool serve = which < nneed;
              const int ts = serve ? wv * 64 + nlist[wv][which] : t;
              float ct[NB];
#pragma unroll
              for (int b = 0; b < NB; ++b) ct[b] = 0.0f;
              if (serve && u < u1) {
                const RecvInfo& rq = recv[ts % nrecv];
                const double qx0 = (double)pd_xj[ts][0], qx1 = (double)pd_xj[ts][1],
                             qx2 = (double)pd_xj[ts][2];
                const double pe0 = qx0 - rq.x[0], pe1 = qx1 - rq.x[1], pe2 = qx2 - rq.x[2];
                const double ux = S.x[u], uy = S.y[u], uz = S.z[u];
                const double f0 = ux - qx0, f1 = uy - qx1, f2 = uz - qx2;
                const double w0 = ux - rq.x[0], w1 = uy - rq.x[1], w2 = uz - rq.x[2];
                double uu = (w0 * pe0 + w1 * pe1 + w2 * pe2) * pd_inv2[ts];
                uu = fmin(1.0, fmax(0.0, uu));
                const double g0 = w0 - uu * pe0, g1 = w1 - uu * pe1, g2 = w2 - uu * pe2;
                const double b2 = g0 * g0 + g1 * g1 + g2 * g2;
                const uint32_t us = S.slot[u];
                if ((f0 * f0 + f1 * f1 + f2 * f2 < pd_r2[ts]) && b2 < S.h2[u] &&
                    us != rq.slot && us != pd_j[ts]) {
                  ++hits;
                  const float bb = __builtin_amdgcn_sqrtf((float)b2);
                  const float sg = S.sig[u] * (1.0f - bb * S.invh[u]);
#pragma unroll
                  for (int b = 0; b < NB; ++b) ct[b] = S.kap[u][b] * sg;
                }
              }
#pragma unroll
              for (int b = 0; b < NB; ++b) ct[b] = group_sum_dpp(ct[b], sub);
              if (serve && u == sb * sub) {
#pragma unroll
                for (int b = 0; b < NB; ++b) tacc[ts][b] += ct[b];
              }
            }
            wave_lds_sync();
            continue;
          }
          if (!need) continue;
          for (int u = sb * sub; u < u1; ++u) {
            const double ux = S.x[u], uy = S.y[u], uz = S.z[u];
            const double f0 = ux - xj0, f1 = uy - xj1, f2 = uz - xj2;
            const double w0 = ux - xi0, w1 = uy - xi1, w2 = uz - xi2;
            double uu = (w0 * e0 + w1 * e1 + w2 * e2) * inv2;
            uu = fmin(1.0, fmax(0.0, uu));
            const double g0 = w0 - uu * e0, g1 = w1 - uu * e1, g2 = w2 - uu * e2;
            const double b2 = g0 * g0 + g1 * g1 + g2 * g2;
            const uint32_t us = S.slot[u];
            if ((f0 * f0 + f1 * f1 + f2 * f2 < rij2) && b2 < S.h2[u] && us != si && us != j) {
              ++hits;
              const float bb = __builtin_amdgcn_sqrtf((float)b2);
              const float sg = S.sig[u] * (1.0f - bb * S.invh[u]);
#pragma unroll
              for (int b = 0; b < NB; ++b) tau[b] += S.kap[u][b] * sg;
            }
          }
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int b = 0; b < NB; ++b) tau[b] += tacc[t][b];
      if (ok) {
        const float Kv = fshape((float)sqrt(rij2) * ri.inv_rh) * ri.kfac;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[b] += (double)T.lum[(int64_t)b * n + j] * (double)Kv * exp(-(double)tau[b]);
          pt[(int64_t)p * NB + b] = tau[b];
        }
      }
    }
    // receiver-wise sums in thread order (deterministic); red shares its LDS
    // with the last pass's tile or queues
    if (hits) atomicAdd(&s_hits, (unsigned long long)hits);
    if (lane == 0 && logn) atomicAdd(&s_logn, (unsigned long long)logn);
    hits = 0;
    logn = 0;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) red[t][b] = acc[b];
    __syncthreads();
    if (J && t < nrecv * NB) {
      const int ii = t / NB, b = t % NB;
      double v = 0.0;
      for (int u = ii; u < stride; u += nrecv) v += red[u][b];
      J[(int64_t)b * n + T.perm[recv[ii].slot]] = v;
    }
  }
  if (J && t == 0) {
    if (T.counters != cdst) {
      pp_counters_flush(cdst, csum);
      cdst = T.counters;
    }
    csum[0] += (unsigned long long)nact * nnear;
    csum[1] += (unsigned long long)nact * nl * nnear;
    csum[2] = max(csum[2], (unsigned long long)nnear);
    csum[3] += s_hits;
    csum[4] += s_logn;
  }
  if (t == 0) {
    s_hits = 0ull;
    s_logn = 0ull;
  }
  if (JL.log) {
    // the bucket's stream starts, or none when the log does not cover it
    if (lane == 0 && (lbeg.blk == kLogNone || lp.blk == kLogNone)) s_logbad = 1u;
    __syncthreads();
    if (lane == 0) JL.tab[4 * bucket + wv] = make_uint2(s_logbad ? kLogNone : lbeg.blk, lbeg.pos);
  }
  }
  if (Jall && threadIdx.x == 0) pp_counters_flush(cdst, csum);
}

// ------------------------------------------------------------- far field
// Adds a workgroup's sums of the far field's per-bucket counters to a
// scene's counters (none when dst is null) and clears them.  Thread 0 keeps
// the sums in LDS across its workgroup's buckets and adds them when it turns
// to another scene and after its last bucket: the counters share a cache
// line, so a set of atomics per bucket queued behind one another.
constexpr int kFarCounters = 6;
__device__ inline void far_counters_flush(unsigned long long* dst, unsigned long long* s) {
  const int slot[kFarCounters] = {CNT_BUCKETS, CNT_CELLS, CNT_ABS, CNT_SRC, CNT_SEG, CNT_SRC_PAIRS};
#pragma unroll
  for (int k = 0; k < kFarCounters; ++k) {
    if (dst && s[k]) atomicAdd(&dst[slot[k]], s[k]);
    s[k] = 0ull;
  }
}

// One workgroup of kFT threads per bucket.  Rays are taken in groups of 64;
// thread k < 64 owns ray k of the group for the per-ray sort and the suffix
// sums; hits are found and applied by whichever thread holds the cut entry.
// Sources of a group are held kSrcCap at a time (a second window re-reads
// the cut; only source-rich buckets need it).  Receivers are fixed per
// thread (t mod P2, P2 the power of two >= the receiver count), so each
// thread keeps one FP64 accumulator per band, reduced per receiver in a
// fixed order at the end.
//
// Workgroups per CU to compile for: as many as the kernel's LDS lets reside
// (up to 4; its LDS grows with the band count, and the source window SrcCap
// is sized for four up to five bands), the register budget capped to match.
// Latency-bound: four workgroups with some spilling beat two without (2^21
// diffuse, two bands: 146 -> 93 ms; clumpy, three bands: 5.8 -> 4.2 ms).
template <int NB> struct FarCfg {
  static constexpr int waves = NB <= 5 ? 4 : NB == 6 ? 3 : NB <= 12 ? 2 : 1;
};

template <int NB>
__global__ void __launch_bounds__(kFT, FarCfg<NB>::waves) k_far(const DevTree* __restrict__ TT, Items I,
                                             const uint32_t* blist, const uint32_t* bscene,
                                             const double* brad, const uint32_t* toff,
                                             const uint2* cut, uint32_t cut_cap,
                                             const uint32_t* bstat, const float* tppg,
                                             const float* bgall, double* Jall,
                                             const uint8_t* active, float* kept_tau,
                                             float* kept_tex) {
  constexpr int kSrcCap = SrcCap<NB>::value;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

  __shared__ SrcWindow<kSrcCap, NB> W;
  __shared__ RayGroup G;
  __shared__ float tpp[kRMax][64][NB];
  __shared__ float tex[64][NB];
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, wcnt[kFT / 64], abs_count, s_item;
  __shared__ double red[kFT / 64][kRMax][NB];
  __shared__ uint32_t hitq[kFT / 64][kHitQ];   // per wavefront: queued (entry, ray) tests
  __shared__ unsigned long long csum[kFarCounters];
  __shared__ unsigned long long* cdst;

  if (threadIdx.x == 0) {
    cdst = nullptr;
    far_counters_flush(nullptr, csum);
  }
  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  double* J = Jall + T.joff;
  const float* bg = bgall ? bgall + T.boff : nullptr;
  const uint32_t rel = bucket - I.lo;
  const uint32_t leafb = blist[bucket];
  const double r = brad[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t ncut = min(bstat[4 * bucket + 0], cut_cap);
  const uint2* mycut = cut + (size_t)rel * cut_cap;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  const int ngroups = (nray + 63) / 64;
  const int64_t n = T.n;
  const bool use_bg = (T.flags & TREVR_BACKGROUND) && bg != nullptr;

  if (t == 0) abs_count = 0u;
  uint32_t nact_total = 0;
  const float* tppb = tppg + toff[bucket];
  uint32_t ract = 0;
  uint32_t member = lk.x;
  for (;;) {
    const int nrecv = load_receivers(T, act, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    const bool first_chunk = nact_total == 0;
    nact_total += (uint32_t)nrecv;
    int P2 = 1;
    while (P2 < nrecv) P2 <<= 1;
    const int my_i = t & (P2 - 1);             // this thread's receiver
    const bool has_i = my_i < nrecv;
    const int per_round = kFT / P2;
    const int my_q = t / P2;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;

    for (int g = 0; g < ngroups; ++g) {
      const int k0 = 64 * g;
      const int kn = min(64, nray - k0);
      const bool rt = t < kn;                  // ray-owning thread
      load_ray_group(T, c, k0, kn, G);
      for (int q = t; q < nrecv * kn; q += kFT) {
        const int i = q / kn, kq = q % kn;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          tpp[i][kq][b] = tppb[((int64_t)(ract + i) * nray + k0 + kq) * NB + b];
      }

      for (uint32_t skip = 0;; skip += (uint32_t)kSrcCap) {
        if (t < 64) {
#pragma unroll
          for (int b = 0; b < NB; ++b) tex[t][b] = 0.0f;
        }
        const uint32_t nsg_all =
            stage_window<kSrcCap, NB>(T, mycut, ncut, c, k0, kn, skip, W, wcnt, nullptr);
        const uint32_t nsg = min(nsg_all - skip, (uint32_t)kSrcCap);
        uint32_t q0, q1;
        sort_window<kSrcCap, NB>(W, nsg, rt, q0, q1);

        // ---- cell absorption along each ray (Sections 2.5.1, 2.6).  Each
        // hit is applied by the thread that found it: sources on its ray
        // inside the chord get the partial length, the nearest source beyond
        // it a suffix add (resolved by a prefix sum over the ray's sources
        // sorted by distance).  The LDS atomics make the FP32 sums depend on
        // the order of the hits at the level of rounding.
        uint32_t nabs = 0;
        for_each_hit_queued(T, mycut, ncut, c, r, kn, G, hitq[wv],
                          [&](uint32_t node, int kq, double ht0, double ht1, bool) {
          const float len = (float)(ht1 - ht0);
          const float* al = &T.alpha[((int64_t)node * T.nclass + G.cls[kq]) * NB];
          float av[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            av[b] = al[b];
            if (use_bg) atomicAdd(&tex[kq][b], av[b] * len);
          }
          ++nabs;
          const uint32_t r0 = W.ray_beg[kq], r1 = W.ray_beg[kq + 1];
          uint32_t lo_p = r0, hi_p = r1;     // first source beyond t0
          while (lo_p < hi_p) {
            const uint32_t mid = (lo_p + hi_p) >> 1;
            if ((double)W.s[W.order[mid]] > ht0) hi_p = mid; else lo_p = mid + 1;
          }
          uint32_t pq = lo_p;
          for (; pq < r1; ++pq) {
            const uint32_t si = W.order[pq];
            const double sq = (double)W.s[si];
            if (!(sq < ht1)) break;
            const float part = (float)(sq - ht0);
#pragma unroll
            for (int b = 0; b < NB; ++b) atomicAdd(&W.tau[si][b], av[b] * part);
          }
          if (pq < r1) {
            const uint32_t si = W.order[pq];
#pragma unroll
            for (int b = 0; b < NB; ++b) atomicAdd(&W.sfx[si][b], av[b] * len);
          }
        });
        if (skip == 0 && first_chunk && nabs) atomicAdd(&abs_count, nabs);
        __syncthreads();
        if (rt) {   // resolve the suffix adds along each ray
          float run[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) run[b] = 0.0f;
          for (uint32_t pq = q0; pq < q1; ++pq) {
            const uint32_t si = W.order[pq];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              run[b] += W.sfx[si][b];
              W.tau[si][b] += run[b];
            }
          }
        }
        __syncthreads();
        // keep the optical depths for the adjoint when the group fits one
        // window (of this kernel and of the adjoint)
        if (kept_tau && first_chunk && nsg_all <= (uint32_t)KeptCap<NB>::value) {
          float* dst = kept_tau + ((size_t)rel * ngroups + g) * KeptCap<NB>::value * NB;
          for (uint32_t q = t; q < nsg * NB; q += kFT) dst[q] = (&W.tau[0][0])[q];
          if (use_bg && t < kn) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
              kept_tex[((size_t)rel * nray + k0 + t) * NB + b] = tex[t][b];
          }
        }

        // ---- far sources at every receiver (Section 2.5.1, eq. intint)
        if (has_i) {
          const RecvInfo& ri = recv[my_i];
          for (uint32_t q = (uint32_t)my_q; q < nsg; q += (uint32_t)per_round) {
            const float dx = W.rel[q][0] - ri.rel[0];
            const float dy = W.rel[q][1] - ri.rel[1];
            const float dz = W.rel[q][2] - ri.rel[2];
            const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
            const float Kv = fshape(rr * ri.inv_rh) * ri.kfac;
            const int ray = W.ray[q];
            // true over projected distance of the source (W.s ends the cell
            // trace, shorter than the projection with the complex source model)
            const float sproj = T.csrc_d ? W.rel[q][0] * G.nf[ray][0] + W.rel[q][1] * G.nf[ray][1] +
                                               W.rel[q][2] * G.nf[ray][2]
                                         : W.s[q];
            const float ratio = rr * __builtin_amdgcn_rcpf(sproj);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const float tau = W.tau[q][b];
              const float tc = (tau > 0.0f) ? tau * ratio : 0.0f;
              const float e = __expf(-(tpp[my_i][ray][b] + tc));
              acc[b] += (double)(W.L[q][b] * Kv * e);
            }
          }
          // ---- isotropic background along each ray (to the root-cube edge)
          if (use_bg && skip == 0) {
            for (int kq = my_q; kq < kn; kq += per_round)
#pragma unroll
              for (int b = 0; b < NB; ++b)
                acc[b] += (4.0 * kPi / nray) * (double)bg[b] *
                          (double)__expf(-(tpp[my_i][kq][b] + tex[kq][b]));
          }
        }
        __syncthreads();
        if (nsg_all <= skip + (uint32_t)kSrcCap) break;
      }
    }

    // ---- per-receiver sums in a fixed order, add the p-p part, thick factor
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = acc[b];
      for (int o = 32; o >= P2 && o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane < P2 && lane < nrecv) red[wv][lane][b] = v;
    }
    __syncthreads();
    if (t < nrecv * NB) {
      const int i = t / NB, b = t % NB;
      double v = 0.0;
      for (int w = 0; w < kFT / 64; ++w) v += red[w][i][b];
      const uint32_t sl = recv[i].slot;
      const int64_t o = (int64_t)b * n + T.perm[sl];
      double out = J[o] + v;
      if (T.flags & TREVR_THICK_CORR) {
        const double tau = (double)T.kappa[(int64_t)b * n + sl] * (double)T.rho[sl] * recv[i].h;
        out *= (tau == 0.0) ? 1.0 : -expm1(-tau) / tau;
      }
      J[o] = out;
    }
    ract += (uint32_t)nrecv;
  }

  __syncthreads();
  if (t == 0) {
    const uint32_t nsrc = bstat[4 * bucket + 1], ncells = bstat[4 * bucket + 2];
    const uint32_t nabs_total = abs_count;
    if (T.counters != cdst) {
      far_counters_flush(cdst, csum);
      cdst = T.counters;
    }
    csum[0] += 1ull;
    csum[1] += (unsigned long long)ncells;
    csum[2] += (unsigned long long)nabs_total;
    csum[3] += (unsigned long long)nsrc;
    csum[4] += (unsigned long long)nact_total * ((unsigned long long)nray + nabs_total + nsrc);
    csum[5] += (unsigned long long)nact_total * nsrc;
  }
  }
  if (threadIdx.x == 0) far_counters_flush(cdst, csum);
}

// ----------------------------------------------------- bucket ordering
// Buckets are grouped by their scene's band count (one launch per count)
// and, within a group, processed heaviest first (a counting sort by the log2
// of an estimate of their p-p work), so the slowest buckets start early
// instead of forming the tail of a launch; or (ORDER_SCENE) scene by scene,
// heaviest first within each, which keeps a scene's tree in the caches.
// Each bucket's result is independent of its position.
// Heaviest-first order bins, counted per workgroup in LDS (one global add
// per workgroup and bin) so the few hot bins are not serialised.
constexpr int kLocalBins = kMaxBands * kCostBins;
__device__ inline int local_bin(uint32_t bin) {
  return (int)(bin / kOrderBins) * kCostBins + (int)(bin % kOrderBins);
}

__global__ void __launch_bounds__(256) k_cost_bins(const DevTree* __restrict__ TT,
                                                   const uint32_t* nbp, const uint32_t* bscene,
                                                   const uint32_t* bnact, const uint32_t* ncnt,
                                                   const uint32_t* nlumc, uint32_t order,
                                                   uint32_t nscenes, uint32_t* bbin,
                                                   uint32_t* bins) {
  __shared__ uint32_t lcnt[kLocalBins];
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  const bool local = order == ORDER_COST;
  if (local)
    for (int i = threadIdx.x; i < kLocalBins; i += blockDim.x) lcnt[i] = 0u;
  __syncthreads();
  if (b < *nbp) {
  const uint32_t sc = bscene[b];
  const DevTree& T = TT[sc];
  const unsigned long long cost =
      (unsigned long long)bnact[b] * ((unsigned long long)ncnt[b] * (T.nray / 2 + nlumc[b]) + 2000ull);
  const int lg = 63 - __clzll((long long)cost);
  uint32_t key = (uint32_t)max(0, (kCostBins - 1) - min(lg, kCostBins - 1));
  if (order == ORDER_SCENE) {   // scene groups in input order, heaviest first inside
    constexpr uint32_t kGroups = kOrderBins / kCostBins;
    key += (uint32_t)((unsigned long long)sc * kGroups / nscenes) * kCostBins;
  }
  const uint32_t bin = (uint32_t)(T.B - 1) * kOrderBins + key;
  bbin[b] = bin;
  if (local) atomicAdd(&lcnt[local_bin(bin)], 1u);
  else atomicAdd(&bins[bin], 1u);
  }
  if (local) {
    __syncthreads();
    for (int i = threadIdx.x; i < kLocalBins; i += blockDim.x)
      if (lcnt[i]) atomicAdd(&bins[(i / kCostBins) * kOrderBins + i % kCostBins], lcnt[i]);
  }
}

// After the exclusive scan of the bins: rng[2 + 2c], rng[3 + 2c] get the
// range of the buckets with c + 1 bands.
__global__ void k_class_ranges(const uint32_t* bins, uint32_t* rng) {
  const int cl = threadIdx.x;
  if (cl >= kMaxBands) return;
  rng[2 + 2 * cl] = bins[cl * kOrderBins];
  rng[3 + 2 * cl] = cl + 1 < kMaxBands ? bins[(cl + 1) * kOrderBins] : rng[1];
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o);
  return v;
}

// Per-bucket sizes of the dynamic scratch, in the processing order: p-p list
// entries (ncnt), p-p column floats (tcnt = receivers x rays x bands), raw-J
// words of the adjoint (jcnt = receivers x bands) and (receiver, luminous p-p
// element) pair floats (pcnt = receivers x luminous x bands); their 64-bit
// totals go to tot[0..3], the receivers to tot[4].
__global__ void __launch_bounds__(256) k_reorder(const DevTree* __restrict__ TT,
                                                 const uint32_t* nbp, uint32_t order,
                                                 const uint32_t* bbin, uint32_t* bins,
                                                 const uint32_t* blist,
                          const uint32_t* bscene, const uint32_t* bnact, const uint32_t* ncnt,
                          const uint32_t* nlumc, const double* brad, const double* bprev,
                          const uint32_t* barg, uint32_t* bsrc2, uint32_t* blist2,
                          uint32_t* bscene2,
                          uint32_t* bnact2, uint32_t* ncnt2, uint32_t* nlumc2, double* brad2,
                          double* bprev2, uint32_t* barg2, uint32_t* tcnt2,
                          uint32_t* jcnt2, uint32_t* pcnt2, unsigned long long* tot) {
  __shared__ uint32_t lcnt[kLocalBins], lbase[kLocalBins];
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  const bool local = order == ORDER_COST;
  const bool valid = b < *nbp;
  // positions: a rank within the workgroup's share of each bin, that share
  // reserved with one global add per bin
  uint32_t rank = 0u;
  if (local) {
    for (int i = threadIdx.x; i < kLocalBins; i += blockDim.x) lcnt[i] = 0u;
    __syncthreads();
    if (valid) rank = atomicAdd(&lcnt[local_bin(bbin[b])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kLocalBins; i += blockDim.x)
      if (lcnt[i]) lbase[i] = atomicAdd(&bins[(i / kCostBins) * kOrderBins + i % kCostBins], lcnt[i]);
    __syncthreads();
  }
  unsigned long long v[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
  if (valid) {
    const uint32_t pos = local ? lbase[local_bin(bbin[b])] + rank : atomicAdd(&bins[bbin[b]], 1u);
    const uint32_t sc = bscene[b];
    const DevTree& T = TT[sc];
    const uint32_t na = bnact[b], B = (uint32_t)T.B;
    bsrc2[pos] = b;
    blist2[pos] = blist[b];
    bscene2[pos] = sc;
    bnact2[pos] = na;
    ncnt2[pos] = ncnt[b];
    nlumc2[pos] = nlumc[b];
    brad2[pos] = brad[b];
    bprev2[pos] = bprev[b];
    barg2[pos] = barg[b];
    tcnt2[pos] = na * (uint32_t)T.nray * B;
    jcnt2[pos] = na * B;
    pcnt2[pos] = na * nlumc[b] * B;
    v[0] = ncnt[b];
    v[1] = (unsigned long long)na * T.nray * B;
    v[2] = (unsigned long long)na * nlumc[b] * B;
    v[3] = (unsigned long long)na * B;
    v[4] = na;
  }
  // per-workgroup sums, then one atomic per total (the totals share a cache
  // line, so every atomic on them queues behind the others)
  __shared__ unsigned long long part[4][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const unsigned long long s = wave_sum_u64(v[k]);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const unsigned long long s = part[0][threadIdx.x] + part[1][threadIdx.x] +
                                 part[2][threadIdx.x] + part[3][threadIdx.x];
    if (s) atomicAdd(&tot[threadIdx.x], s);
  }
}

// ============================================================ host side
__global__ void k_zero_words(uint32_t* a, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) a[i] = 0u;
}

static unsigned grid_of(int64_t work, int threads) {
  return (unsigned)std::max<int64_t>(1, (work + threads - 1) / threads);
}

#define TREVR_LAUNCH_CHECK(what)                                               \
  do {                                                                         \
    if ((rc = hip_check(hipGetLastError(), what)) != TREVR_OK) return rc;      \
  } while (0)

trevr_status zero_words(hipStream_t st, void* p, size_t words) {
  trevr_status rc = TREVR_OK;
  if (words == 0) return rc;
  k_zero_words<<<grid_of((int64_t)words, 256), 256, 0, st>>>((uint32_t*)p, (int64_t)words);
  TREVR_LAUNCH_CHECK("k_zero_words");
  return rc;
}

size_t default_cut_entries(int64_t leaves) {
  return (size_t)std::min<int64_t>(std::max<int64_t>(leaves, 1), kBatch) * kCutCap;
}

Scratch carve_scratch(void* base, int64_t leaves, size_t cut_entries) {
  Carve cv(base);
  Scratch s{};
  const int64_t L = std::max<int64_t>(leaves, 1);
  s.rng = cv.take<uint32_t>(2 + 2 * kMaxBands);
  s.q = cv.take<uint32_t>(2 * Q_N);
  s.tot = cv.take<unsigned long long>(TOT_N);
  s.ovf = cv.take<uint32_t>(4);
  s.ahash = cv.take<unsigned long long>(2);
  s.bins = cv.take<uint32_t>(kMaxBands * kOrderBins);
  s.ncnt = cv.take<uint32_t>(L + 1);
  s.tcnt = cv.take<uint32_t>(L + 1);
  s.jcnt = cv.take<uint32_t>(L + 1);
  s.pcnt = cv.take<uint32_t>(L + 1);
  s.zero_words = (cv.off - (size_t)((char*)s.rng - (char*)base)) / 4;
  s.blist = cv.take<uint32_t>(L);
  s.bscene = cv.take<uint32_t>(L);
  s.bnact = cv.take<uint32_t>(L);
  s.nlumc = cv.take<uint32_t>(L);
  s.bstat = cv.take<uint32_t>(4 * L);
  s.brad = cv.take<double>(L);
  s.bprev = cv.take<double>(L);
  s.barg = cv.take<uint32_t>(L);
  s.bsrc = cv.take<uint32_t>(L);
  s.blist_raw = cv.take<uint32_t>(L);
  s.bscene_raw = cv.take<uint32_t>(L);
  s.bnact_raw = cv.take<uint32_t>(L);
  s.ncnt_raw = cv.take<uint32_t>(L);
  s.nlumc_raw = cv.take<uint32_t>(L);
  s.bbin = cv.take<uint32_t>(L);
  s.brad_raw = cv.take<double>(L);
  s.bprev_raw = cv.take<double>(L);
  s.barg_raw = cv.take<uint32_t>(L);
  s.cut_entries = cut_entries;
  s.cut = cv.take<uint2>(cut_entries);
  s.stage = reinterpret_cast<uint32_t*>(s.cut);
  const size_t per = std::min<size_t>(kStageCap, 2 * cut_entries / (size_t)L) & ~(size_t)63;
  s.stage_cap = (uint32_t)per;
  s.fixed = ((cv.off + 255) & ~(size_t)255) + 256;   // 256-aligned
  return s;
}

Launch tree_launch(const trevr_tree* T) {
  return Launch{T->stream, T->buf.dev, 1, T->num_nodes, T->n, T->num_leaves, T->stack_large,
                LaunchCfg{}};
}

unsigned persistent_grid(const void* fn, int threads, uint64_t items, uint32_t div) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> occ;
  static std::unordered_map<int, int> cus;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int per_cu = 0, ncu = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = occ.find(fn);
    if (it == occ.end()) {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, threads, 0) != hipSuccess || b < 1)
        b = 1;
      it = occ.emplace(fn, b).first;
    }
    per_cu = it->second;
    auto jt = cus.find(dev);
    if (jt == cus.end()) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          v < 1)
        v = 1;
      jt = cus.emplace(dev, v).first;
    }
    ncu = jt->second;
  }
  const uint64_t slots = std::max<uint64_t>(1, (uint64_t)per_cu * (uint64_t)ncu / std::max(div, 1u));
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(items, slots));
}

// Cell optical depths the forward keeps for the adjoint (TREVR_KEEP_DEPTHS):
// per bucket of a batch and ray group, KeptCap sources x bands (and with a
// background the exit depth per ray); not kept without the flag or when that
// would take more than 1 GiB.
void take_kept(const trevr_tree* T, Scratch& S, Carve& cv, uint32_t nb) {
  const size_t buckets = std::min<size_t>(nb, kBatch);
  const size_t groups = (size_t)(T->nray + 63) / 64;
  static constexpr int caps[9] = {0, KeptCap<1>::value, KeptCap<2>::value, KeptCap<3>::value,
                                  KeptCap<4>::value, KeptCap<5>::value, KeptCap<6>::value,
                                  KeptCap<7>::value, KeptCap<8>::value};
  const size_t tau_n = buckets * groups * caps[T->B] * T->B;
  const size_t tex_n = (T->p.flags & TREVR_BACKGROUND) ? buckets * T->nray * T->B : 0;
  if (!(T->p.flags & TREVR_KEEP_DEPTHS) || (tau_n + tex_n) * sizeof(float) > ((size_t)1 << 30)) {
    S.kept_tau = nullptr;
    S.kept_tex = nullptr;
    return;
  }
  S.kept_tau = cv.take<float>(tau_n);
  S.kept_tex = tex_n ? cv.take<float>(tex_n) : nullptr;
}

namespace {
std::mutex g_scratch_mu;
std::unordered_map<const void*, uint64_t> g_scratch_epoch;
uint64_t g_epoch = 0;
}  // namespace

uint64_t scratch_mark(const void* scratch) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_epoch.size() > 4096) g_scratch_epoch.clear();   // only disables reuse
  g_scratch_epoch[scratch] = ++g_epoch;
  return g_epoch;
}

bool scratch_unchanged(const void* scratch, uint64_t epoch) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  const auto it = g_scratch_epoch.find(scratch);
  return it != g_scratch_epoch.end() && it->second == epoch;
}
size_t scratch_fixed_bytes(int64_t n) {
  return carve_scratch(nullptr, n, default_cut_entries(n)).fixed;   // leaves <= n
}

trevr_status setup_kernels(const Launch& L, const uint8_t* active, const Scratch& S) {
  hipStream_t st = L.st;
  trevr_status rc;
  if ((rc = zero_words(st, S.rng, S.zero_words)) != TREVR_OK) return rc;
  const dim3 gn(grid_of(L.max_nodes, 256), (unsigned)L.S);
  k_active_buckets<<<gn, 256, 0, st>>>(L.TT, active, S.blist_raw, S.bscene_raw, S.bnact_raw,
                                       S.rng + 1);
  TREVR_LAUNCH_CHECK("k_active_buckets");
  const Items I{0u, 0xFFFFFFFFu, S.rng, nullptr};
  const unsigned gb = grid_of(L.leaves, 1);
  if (L.stack_large)
    k_setup<kStackLarge><<<gb, 64, 0, st>>>(L.TT, I, S.blist_raw, S.bscene_raw, S.brad_raw,
                                             S.bprev_raw, S.barg_raw, S.ncnt_raw, S.nlumc_raw,
                                             S.ovf, S.stage, S.stage_cap);
  else
    k_setup<kStackSmall><<<gb, 64, 0, st>>>(L.TT, I, S.blist_raw, S.bscene_raw, S.brad_raw,
                                             S.bprev_raw, S.barg_raw, S.ncnt_raw, S.nlumc_raw,
                                             S.ovf, S.stage, S.stage_cap);
  TREVR_LAUNCH_CHECK("k_setup");
  const unsigned gl = grid_of(L.leaves, 256);
  k_cost_bins<<<gl, 256, 0, st>>>(L.TT, S.rng + 1, S.bscene_raw, S.bnact_raw, S.ncnt_raw,
                                  S.nlumc_raw, L.cfg.order, (uint32_t)L.S, S.bbin, S.bins);
  TREVR_LAUNCH_CHECK("k_cost_bins");
  k_scan_u32<<<1, 1024, 0, st>>>(S.bins, (int64_t)kMaxBands * kOrderBins, nullptr);
  TREVR_LAUNCH_CHECK("k_scan_u32");
  k_class_ranges<<<1, 64, 0, st>>>(S.bins, S.rng);
  TREVR_LAUNCH_CHECK("k_class_ranges");
  k_reorder<<<gl, 256, 0, st>>>(L.TT, S.rng + 1, L.cfg.order, S.bbin, S.bins, S.blist_raw,
                                S.bscene_raw, S.bnact_raw, S.ncnt_raw, S.nlumc_raw, S.brad_raw,
                                S.bprev_raw, S.barg_raw, S.bsrc, S.blist, S.bscene, S.bnact,
                                S.ncnt, S.nlumc, S.brad, S.bprev, S.barg, S.tcnt, S.jcnt, S.pcnt,
                                S.tot);
  TREVR_LAUNCH_CHECK("k_reorder");
  const int64_t Lp = std::max<int64_t>(L.leaves, 1) + 1;
  k_scan_arrays<<<4, 1024, 0, st>>>(ScanArrays{{S.ncnt, S.tcnt, S.jcnt, S.pcnt}}, Lp);
  TREVR_LAUNCH_CHECK("k_scan_arrays");
  const dim3 ge(std::min(grid_of(L.max_n, 256), kHashBlocks), (unsigned)L.S);
  k_active_hash<<<ge, 256, 0, st>>>(L.TT, active, S.ahash);
  TREVR_LAUNCH_CHECK("k_active_hash");
  return TREVR_OK;
}

trevr_status launch_active_hash(const Launch& L, const uint8_t* active,
                                unsigned long long* out) {
  trevr_status rc;
  if ((rc = zero_words(L.st, out, 2)) != TREVR_OK) return rc;
  const dim3 ge(std::min(grid_of(L.max_n, 256), kHashBlocks), (unsigned)L.S);
  k_active_hash<<<ge, 256, 0, L.st>>>(L.TT, active, out);
  TREVR_LAUNCH_CHECK("k_active_hash");
  return rc;
}

trevr_status bucket_setup(trevr_tree* T, const uint8_t* active, Scratch& S, uint32_t* nb,
                          uint64_t tot[TOT_N], uint64_t* hash) {
  hipStream_t st = T->stream;
  trevr_status rc;
  uint32_t* hbuf = T->host_u32;
  for (;;) {
    const Launch L = tree_launch(T);
    if ((rc = setup_kernels(L, active, S)) != TREVR_OK) return rc;
    hipError_t e = hipMemcpyAsync(hbuf, S.tot, TOT_N * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hbuf + 2 * TOT_N, S.ahash, sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hbuf + 2 * TOT_N + 2, S.rng + 1, sizeof(uint32_t),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hbuf + 2 * TOT_N + 3, S.ovf, sizeof(uint32_t), hipMemcpyDeviceToHost,
                         st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if ((rc = hip_check(e, "bucket readback")) != TREVR_OK) return rc;
    if (!(hbuf[2 * TOT_N + 3] & OVF_SETUP)) break;
    // a p-p range query ran out of the small traversal stack: use the
    // large one for this tree from now on
    if (T->stack_large)
      return set_error(TREVR_E_CAPACITY, "a p-p range query exceeds the traversal stack");
    T->stack_large = true;
  }
  std::memcpy(tot, hbuf, TOT_N * sizeof(uint64_t));
  std::memcpy(hash, hbuf + 2 * TOT_N, sizeof(uint64_t));
  *nb = hbuf[2 * TOT_N + 2];
  for (int k = 0; k < TOT_RECV; ++k)
    if (tot[k] > 0xFFFFFFFFull)
      return set_error(TREVR_E_CAPACITY, "per-call p-p sizes exceed 32-bit offsets");
  return TREVR_OK;
}

trevr_status active_hash(trevr_tree* T, const uint8_t* active, unsigned long long* dev_slot,
                         uint64_t* hash) {
  hipStream_t st = T->stream;
  trevr_status rc;
  if ((rc = zero_words(st, dev_slot, 2)) != TREVR_OK) return rc;
  const dim3 ge(std::min(grid_of(T->n, 256), kHashBlocks), 1u);
  k_active_hash<<<ge, 256, 0, st>>>(T->buf.dev, active, dev_slot);
  TREVR_LAUNCH_CHECK("k_active_hash");
  uint32_t* hbuf = T->host_u32;
  hipError_t e = hipMemcpyAsync(hbuf + 2 * TOT_N, dev_slot, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if ((rc = hip_check(e, "hash readback")) != TREVR_OK) return rc;
  std::memcpy(hash, hbuf + 2 * TOT_N, sizeof(uint64_t));
  return TREVR_OK;
}

trevr_status near_fill(const Launch& L, const Scratch& S) {
  trevr_status rc = TREVR_OK;
  const unsigned g = grid_of(L.leaves, 1);
  if (L.stack_large)
    k_near_fill<kStackLarge><<<g, 64, 0, L.st>>>(L.TT, S.rng, S.blist, S.bscene, S.brad, S.ncnt,
                                                  S.nlumc, S.bsrc, S.stage, S.stage_cap, S.nidx);
  else
    k_near_fill<kStackSmall><<<g, 64, 0, L.st>>>(L.TT, S.rng, S.blist, S.bscene, S.brad, S.ncnt,
                                                  S.nlumc, S.bsrc, S.stage, S.stage_cap, S.nidx);
  TREVR_LAUNCH_CHECK("k_near_fill");
  return rc;
}

trevr_status walk_launch(const Launch& L, const Scratch& S, const Items& I, uint64_t count,
                         uint32_t cap) {
  trevr_status rc;
  if ((rc = zero_words(L.st, S.ovf, 2)) != TREVR_OK) return rc;
  const unsigned gb = grid_of((int64_t)count, 1);
  if (L.stack_large)
    k_walk<kStackLarge><<<gb, 64, 0, L.st>>>(L.TT, I, S.blist, S.bscene, S.brad, S.cut, cap,
                                              S.bstat, S.ovf);
  else
    k_walk<kStackSmall><<<gb, 64, 0, L.st>>>(L.TT, I, S.blist, S.bscene, S.brad, S.cut, cap,
                                              S.bstat, S.ovf);
  TREVR_LAUNCH_CHECK("k_walk");
  return rc;
}

trevr_status walk_batch(trevr_tree* T, const Scratch& S, uint32_t b0, uint32_t cnt,
                        const std::function<trevr_status(uint32_t, uint32_t, uint32_t)>& run,
                        bool* whole) {
  trevr_status rc;
  uint32_t* hbuf = T->host_u32;
  for (;;) {
    hipEvent_t ev = prof_begin(T);
    if ((rc = walk_launch(tree_launch(T), S, Items{b0, b0 + cnt, nullptr, nullptr}, cnt,
                          T->cut_default)) != TREVR_OK)
      return rc;
    prof_end(T, TREVR_PROF_WALK, ev);
    hipError_t e = hipMemcpyAsync(hbuf, S.ovf, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  T->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
    if ((rc = hip_check(e, "walk readback")) != TREVR_OK) return rc;
    if (!(hbuf[0] & OVF_WALK)) break;
    if (T->stack_large) return set_error(TREVR_E_CAPACITY, "a tree walk exceeds the traversal stack");
    T->stack_large = true;
  }
  const uint32_t maxcut = hbuf[1];
  if (maxcut <= T->cut_default) {
    *whole = true;
    return run(b0, cnt, T->cut_default);
  }
  // some bucket needs a longer cut list: walk the batch again in parts that
  // fit the cut buffer with room for the longest
  *whole = false;
  const size_t cap2 = ((size_t)maxcut + 255) & ~(size_t)255;
  if (cap2 > S.cut_entries)
    return set_error(TREVR_E_CAPACITY, "a bucket's cut list exceeds the cut-list buffer");
  const uint32_t per = (uint32_t)std::max<size_t>(1, S.cut_entries / cap2);
  for (uint32_t s0 = b0; s0 < b0 + cnt; s0 += per) {
    const uint32_t scnt = std::min<uint32_t>(per, b0 + cnt - s0);
    hipEvent_t ev = prof_begin(T);
    if ((rc = walk_launch(tree_launch(T), S, Items{s0, s0 + scnt, nullptr, nullptr}, scnt,
                          (uint32_t)cap2)) != TREVR_OK)
      return rc;
    prof_end(T, TREVR_PROF_WALK, ev);
    if ((rc = run(s0, scnt, (uint32_t)cap2)) != TREVR_OK) return rc;
  }
  return TREVR_OK;
}

template <int NB>
static trevr_status pp_rays_nb(const Launch& L, const Scratch& S, const Items& I, uint64_t count,
                               const uint8_t* active) {
  trevr_status rc;
  const void* fn = (const void*)&k_pp_rays<NB>;
  k_pp_rays<NB><<<persistent_grid(fn, kNT, count, L.cfg.grid_div), kNT, 0, L.st>>>(
      L.TT, I, S.blist, S.bscene, S.ncnt, S.nidx, S.tcnt, active, S.tpp);
  TREVR_LAUNCH_CHECK("k_pp_rays");
  return rc;
}

template <int NB>
static trevr_status pp_src_nb(const Launch& L, const Scratch& S, const Items& I, uint64_t count,
                              const uint8_t* active, double* J) {
  trevr_status rc;
  const void* fn = (const void*)&k_pp_src<NB>;
  k_pp_src<NB><<<persistent_grid(fn, kNT, count, L.cfg.grid_div), kNT, 0, L.st>>>(
      L.TT, I, S.blist, S.bscene, S.ncnt, S.nlumc, S.nidx, S.pcnt, active, J, S.ptau,
      L.cfg.pp_sub, S.jlog);
  TREVR_LAUNCH_CHECK("k_pp_src");
  return rc;
}

template <int NB>
static trevr_status far_nb(const Launch& L, const Scratch& S, const Items& I, uint64_t count,
                           uint32_t cap, const float* bg, double* J, const uint8_t* active) {
  trevr_status rc;
  const void* fn = (const void*)&k_far<NB>;
  k_far<NB><<<persistent_grid(fn, kFT, count, L.cfg.grid_div), kFT, 0, L.st>>>(
      L.TT, I, S.blist, S.bscene, S.brad, S.tcnt, S.cut, cap, S.bstat, S.tpp, bg, J, active,
      S.kept_tau, S.kept_tex);
  TREVR_LAUNCH_CHECK("k_far");
  return rc;
}

#define TREVR_BAND_SWITCH(B, call)              \
  switch (B) {                                  \
    case 1: { constexpr int NB = 1; return call; } \
    case 2: { constexpr int NB = 2; return call; } \
    case 3: { constexpr int NB = 3; return call; } \
    case 4: { constexpr int NB = 4; return call; } \
    case 5: { constexpr int NB = 5; return call; } \
    case 6: { constexpr int NB = 6; return call; } \
    case 7: { constexpr int NB = 7; return call; } \
    case 8: { constexpr int NB = 8; return call; } \
    case 9: { constexpr int NB = 9; return call; } \
    case 10: { constexpr int NB = 10; return call; } \
    case 11: { constexpr int NB = 11; return call; } \
    case 12: { constexpr int NB = 12; return call; } \
    case 13: { constexpr int NB = 13; return call; } \
    case 14: { constexpr int NB = 14; return call; } \
    case 15: { constexpr int NB = 15; return call; } \
    default: { constexpr int NB = 16; return call; } \
  }

trevr_status launch_pp_rays(const Launch& L, int B, const Scratch& S, const Items& I,
                            uint64_t count, const uint8_t* active) {
  TREVR_BAND_SWITCH(B, pp_rays_nb<NB>(L, S, I, count, active))
}

trevr_status launch_pp_src(const Launch& L, int B, const Scratch& S, const Items& I,
                           uint64_t count, const uint8_t* active, double* J) {
  TREVR_BAND_SWITCH(B, pp_src_nb<NB>(L, S, I, count, active, J))
}

trevr_status launch_far(const Launch& L, int B, const Scratch& S, const Items& I,
                        uint64_t count, uint32_t cap, const float* bg, double* J,
                        const uint8_t* active) {
  TREVR_BAND_SWITCH(B, far_nb<NB>(L, S, I, count, cap, bg, J, active))
}
#undef TREVR_BAND_SWITCH

trevr_status compute_J_impl(trevr_tree* T, const uint8_t* active, const float* bg, double* J,
                            void* scratch, size_t scratch_bytes) {
  hipStream_t st = T->stream;
  Scratch S = carve_scratch(scratch, T->num_leaves, default_cut_entries(T->num_leaves));
  S.stage_cap = std::min(S.stage_cap, T->stage_limit & ~63u);
  if (scratch_bytes < S.fixed) {
    T->scratch_needed = S.fixed;
    return set_error(TREVR_E_CAPACITY, "scratch smaller than its fixed part");
  }
  trevr_status rc;
  T->fwd.valid = false;
  const uint64_t epoch = scratch_mark(scratch);
  if ((rc = zero_words(st, T->buf.counters, 2 * CNT_N)) != TREVR_OK) return rc;
  hipEvent_t ev_setup = prof_begin(T);
  uint32_t nb = 0;
  uint64_t tot[TOT_N];
  uint64_t hash = 0;
  if ((rc = bucket_setup(T, active, S, &nb, tot, &hash)) != TREVR_OK) return rc;
  Carve dyn((char*)scratch + S.fixed);
  S.nidx = dyn.take<uint32_t>(tot[TOT_NEAR]);
  S.tpp = dyn.take<float>(tot[TOT_TPP]);
  S.ptau = dyn.take<float>(tot[TOT_PTAU]);
  take_kept(T, S, dyn, nb);
  const size_t need = S.fixed + dyn.off + 256;
  T->scratch_needed = need;
  if (scratch_bytes < need) return set_error(TREVR_E_CAPACITY, "scratch too small for the p-p lists");
  if ((rc = near_fill(tree_launch(T), S)) != TREVR_OK) return rc;
  prof_end(T, TREVR_PROF_SETUP, ev_setup);
  bool whole = true;
  for (uint32_t b0 = 0; b0 < nb; b0 += kBatch) {
    const uint32_t cnt = std::min<uint32_t>(kBatch, nb - b0);
    rc = walk_batch(T, S, b0, cnt, [&](uint32_t s0, uint32_t scnt, uint32_t cap) {
      const Launch L = tree_launch(T);
      trevr_status r;
      hipEvent_t e0 = prof_begin(T);
      if ((r = launch_pp_rays(L, T->B, S, host_items(S, Q_PPR, s0, scnt), scnt, active)) !=
          TREVR_OK)
        return r;
      hipEvent_t e2 = prof_begin(T);
      if ((r = launch_pp_src(L, T->B, S, host_items(S, Q_PPS, s0, scnt), scnt, active, J)) !=
          TREVR_OK)
        return r;
      prof_end(T, TREVR_PROF_PP_SRC, e2);
      prof_end(T, TREVR_PROF_NEAR, e0);
      hipEvent_t e1 = prof_begin(T);
      if ((r = launch_far(L, T->B, S, host_items(S, Q_FAR, s0, scnt), scnt, cap, bg, J,
                          active)) != TREVR_OK)
        return r;
      prof_end(T, TREVR_PROF_REDUCE, e1);
      return r;
    }, &whole);
    if (rc != TREVR_OK) return rc;
  }
  T->counters_valid = true;
  T->fwd = FwdState{true, scratch, epoch, hash, nb, tot[TOT_NEAR], tot[TOT_TPP], tot[TOT_PTAU],
                    tot[TOT_JRAW], nb <= kBatch && whole, T->cut_default,
                    S.kept_tau != nullptr && nb <= kBatch && whole};
  return TREVR_OK;
}
#undef TREVR_LAUNCH_CHECK

}  // namespace trevr
