// Device helpers shared by the forward and adjoint kernels of the mean
// intensity path (Sections 2.1-2.6 of Wadsley, Baumschlager & Shen 2023):
// launch constants, wavefront utilities, the p-p range query, the opening
// test, the element intensity kernel, LDS staging of the p-p set, receiver
// chunks and block-wide compaction.  Everything here is inline; the kernels
// that use it live in compute_j.hip (forward) and compute_j_bwd.hip (adjoint).
#pragma once

#include "trevr_internal.hpp"

namespace trevr {
constexpr int kRMax = 8;         // receivers per pass
// Entries of a traversal stack of SC words that a kernel may use: the small
// stack honours the tree's (tunable) limit.
template <int SC> __device__ inline int stack_cap(const DevTree& T) {
  return SC == kStackSmall ? min(SC, T.stack_limit) : SC;
}

// Per-call overflow word (in the scratch): bits of traversals that ran out
// of stack; the host retries those with the large stack.
enum : uint32_t { OVF_SETUP = 1u, OVF_WALK = 2u };
constexpr uint32_t kBatch = 65536;   // buckets per launch (bounds the cut-list scratch)
constexpr int kCostBins = 48;
constexpr int kOrderBins = 4096;   // counting-sort bins per band count
enum : uint32_t { ORDER_COST = 0, ORDER_SCENE = 1 };
constexpr int kNT = 256;         // threads of the near-field kernel
constexpr int kNChunk = 256;     // p-p elements staged per pass
constexpr int kNPair = 2;        // (receiver, p-p source) pairs per thread per pass
constexpr int kRayPer = 2;       // rays per thread in the p-p column pass
constexpr double kR = 0.48860251190291992;   // (3/(4 pi))^(1/2)

// Work items of one launch (active buckets, each with its scene): indices
// [lo, hi), narrowed by the device-resident range rng[0..1] when given, so a
// launch can cover a count only the device knows.  A fixed grid of
// workgroups (as many as are resident on the chip at once) takes the items
// in order through the counter q[0]; q[1] counts the workgroups that found
// none left, and the last of them clears both, so the pair is zero before
// and after every launch (the caller zeroes it once per scratch use).  A plain
// grid launch (grid_item) leaves q unused; it may be null there.
constexpr uint32_t kNoItem = 0xFFFFFFFFu;
struct Items {
  uint32_t lo, hi;
  const uint32_t* rng;
  uint32_t* q;
};

// Next item for the whole workgroup (kNoItem when none is left); a barrier
// first, so the previous item's LDS is free.
__device__ inline uint32_t next_item(const Items& I, uint32_t* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = I.lo, e = I.hi;
    if (I.rng) {
      b = max(b, I.rng[0]);
      e = min(e, I.rng[1]);
    }
    const uint32_t k = atomicAdd(&I.q[0], 1u);
    uint32_t it = kNoItem;
    if (b < e && k < e - b) {
      it = b + k;
    } else if (atomicAdd(&I.q[1], 1u) == gridDim.x - 1u) {
      atomicExch(&I.q[0], 0u);
      atomicExch(&I.q[1], 0u);
    }
    *s_item = it;
  }
  __syncthreads();
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)*s_item);
}

// The item of this workgroup in a plain grid launch of one workgroup per
// item (blockIdx.x counts from the start of the range), kNoItem past its
// end.  The light per-bucket kernels (setup, walk) launch this way: the
// hardware hands out workgroups in order, and a work-queue claim would cost
// them more than it balances.
__device__ inline uint32_t grid_item(const Items& I) {
  uint32_t b = I.lo, e = I.hi;
  if (I.rng) {
    b = max(b, I.rng[0]);
    e = min(e, I.rng[1]);
  }
  const uint32_t it = b + blockIdx.x;
  return (b < e && it < e) ? it : kNoItem;
}

// Queue counter pairs of a scratch, one per item kernel.
enum { Q_PPR = 0, Q_PPS, Q_FAR, Q_PPS_BWD, Q_FAR_BWD, Q_PPR_BWD, Q_N };

// Order LDS writes of some lanes before reads by other lanes of the same
// wavefront (the lanes execute together; this keeps the compiler and the
// memory model from reordering across the hand-off).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The atomic only when v exceeds the value read first (a stale read is never
// larger than the current value, so no update is lost): most callers'
// values stop exceeding the maximum early, and atomics on one address queue.
__device__ inline void atomic_max_u64(unsigned long long* a, unsigned long long v) {
  if (v > __atomic_load_n(a, __ATOMIC_RELAXED)) atomicMax(a, v);
}

__device__ inline void leaf_centre(const DevTree& T, uint32_t leaf, double c[3]) {
  double lo[3], hi[3];
  node_box(T.hdr, T.nk[leaf], lo, hi);
  for (int a = 0; a < 3; ++a) c[a] = 0.5 * (lo[a] + hi[a]);
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline uint32_t wave_min_u(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
// exclusive prefix sum over the wavefront
__device__ inline uint32_t wave_excl(uint32_t v, int lane) {
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)incl, o);
    if (lane >= o) incl += u;
  }
  return incl - v;
}

// Exclusive prefix over the wavefront of v < 2^BITS, from one ballot per
// bit (no cross-lane data movement); *total gets the wavefront's sum.
template <int BITS>
__device__ inline uint32_t wave_excl_bits(uint32_t v, uint32_t* total) {
  uint32_t e = 0, t = 0;
#pragma unroll
  for (int i = 0; i < BITS; ++i) {
    const uint64_t m = ballot64((v >> i) & 1u);
    e += (uint32_t)mbcnt(m) << i;
    t += (uint32_t)__popcll(m) << i;
  }
  *total = t;
  return e;
}

// Square root for the conservative FP32 culling tests: the hardware
// instruction (within about an ulp), far inside their margins; the correctly
// rounded sqrtf expands to a dozen instructions.
__device__ inline float cull_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

constexpr int kLeafBatch = 8;   // leaf elements loaded together by one lane
static_assert(kLeafBatch <= 16, "a run keeps 16 member bits of each kind");
constexpr int kLeafBatchBits = 4;   // bits of a count in [0, kLeafBatch]
static_assert(kLeafBatch < (1 << kLeafBatchBits), "kLeafBatchBits too small");

// Where a range query puts the elements it finds (out == nullptr: nowhere,
// it only counts them).
//  * slots (runs == false): the k-th luminous element found goes to
//    out[lum0 + k], the k-th other one to out[dark0 + k];
//  * runs (runs == true): each lane's members among kLeafBatch consecutive
//    slots of one leaf make one run of two words, {first slot of the window,
//    luminous member bits | other member bits << 16}; the i-th run found
//    goes to out[2 (nrun + i)], and nrun counts the runs written.  A step
//    that would take nrun past cap ends the writing (out becomes null: the
//    set did not fit).
struct NearOut {
  uint32_t* out;
  bool runs;
  uint32_t lum0, dark0;
  uint32_t nrun, cap;
};

// Range query by one wavefront: elements strictly within sqrt(r2) of c.
// Returns the count; *hmax gets their largest size, *nlum the number that
// emit; the elements go where `o` says.  Boxes are pruned conservatively (an
// element can sit an ulp outside its box after quantisation); membership is
// the exact test.  With r2in >= 0, only the shell r2in <= d2 < r2 (cells
// surely inside the inner sphere are skipped), so a sphere that grows can be
// counted shell by shell with the same memberships.  The traversal stack
// lives in `stack` (cap words).
__device__ inline uint32_t wave_near(const DevTree& T, const double c[3], double r2, uint32_t* stack,
                                     int cap, double* hmax, uint32_t* nlum, NearOut& o,
                                     bool* overflow, uint32_t* harg = nullptr,
                                     double r2in = -1.0) {
  const int lane = threadIdx.x & 63;
  const double prune = r2 * (1.0 + 1e-9);
  // cells surely inside the inner sphere (every element d2 < r2in)
  const double inner = r2in * (1.0 - 1e-9) - 1e-12 * T.hdr[3] * T.hdr[3];
  uint32_t cnt = 0, lum = 0, ha = 0xFFFFFFFFu;
  double hm = 0.0;
  int sp = 1, maxsp = 1;
  if (lane == 0) stack[0] = 0u;
  __syncthreads();
  while (sp > 0) {
    const int take = min(sp, 64);
    sp -= take;
    const bool valid = lane < take;
    const uint32_t node = valid ? stack[sp + lane] : 0u;
    __syncthreads();
    bool push = false;
    uint2 lk = make_uint2(0, 0);
    uint32_t len = 0;   // elements of the leaf this lane opened
    if (valid) {
      const uint4 nk = T.nk[node];
      const uint2 nl = T.nlink[node];   // loaded with the key, off the box test's path
      double lo[3], hi[3];
      node_box(T.hdr, nk, lo, hi);
      if (!(dist2_box(lo, hi, c) > prune) && !(far2_box(lo, hi, c) < inner)) {
        const bool isleaf = (nk.w & META_LEAF) != 0u;
        lk = nl;
        push = !isleaf;
        if (isleaf) len = lk.y;
      }
    }
    // the opened leaves' elements, kLeafBatch per lane at a time with the
    // loads issued together, in step across the wavefront (ballots place the
    // writes)
    for (uint32_t s0 = 0; ballot64(s0 < len) != 0ull; s0 += kLeafBatch) {
      float px[kLeafBatch], py[kLeafBatch], pz[kLeafBatch];
      double ph[kLeafBatch], pl[kLeafBatch];
#pragma unroll
      for (int k = 0; k < kLeafBatch; ++k) {
        const uint32_t s = len ? lk.x + min(s0 + (uint32_t)k, len - 1u) : 0u;
        px[k] = T.x[s];
        py[k] = T.y[s];
        pz[k] = T.z[s];
        ph[k] = T.h[s];
        pl[k] = T.lbol[s];
      }
      uint32_t ml = 0, md = 0;   // members of this step that emit / do not
#pragma unroll
      for (int k = 0; k < kLeafBatch; ++k) {
        const uint32_t s = lk.x + s0 + (uint32_t)k;
        const double d2 = dist2_pt3((double)px[k], (double)py[k], (double)pz[k], c);
        if (s0 + (uint32_t)k < len && d2 < r2 && !(d2 < r2in)) {
          const double hs = ph[k];
          if (hs > hm || (hs == hm && s < ha)) {   // smallest slot among equal sizes
            hm = hs;
            ha = s;
          }
          if (pl[k] > 0.0) ml |= 1u << k;
          else md |= 1u << k;
        }
      }
      uint32_t tl, td;
      const uint32_t el = wave_excl_bits<kLeafBatchBits>((uint32_t)__popc(ml), &tl);
      const uint32_t ed = wave_excl_bits<kLeafBatchBits>((uint32_t)__popc(md), &td);
      if (o.out && o.runs) {
        const bool has = (ml | md) != 0u;
        const uint64_t hb = ballot64(has);
        const uint32_t nr = (uint32_t)__popcll(hb);
        if (nr > o.cap - o.nrun) {   // nrun <= cap while writing
          o.out = nullptr;
        } else {
          if (has)
            reinterpret_cast<uint2*>(o.out)[o.nrun + (uint32_t)mbcnt(hb)] =
                make_uint2(lk.x + s0, ml | (md << 16));
          o.nrun += nr;
        }
      } else if (o.out) {
        uint32_t a = o.lum0 + lum + el, b = o.dark0 + (cnt - lum) + ed;
#pragma unroll
        for (int k = 0; k < kLeafBatch; ++k) {
          const uint32_t s = lk.x + s0 + (uint32_t)k;
          if ((ml >> k) & 1u) o.out[a++] = s;
          if ((md >> k) & 1u) o.out[b++] = s;
        }
      }
      cnt += tl + td;
      lum += tl;
    }
    const uint64_t pm = ballot64(push);
    const int npush = __popcll(pm);
    if (sp + 2 * npush > cap) {
      *overflow = true;
      break;
    }
    if (push) {
      const int ppos = mbcnt(pm);
      stack[sp + 2 * ppos] = lk.x;          // child 1
      stack[sp + 2 * ppos + 1] = node + 1u; // child 0
    }
    sp += 2 * npush;
    maxsp = max(maxsp, sp);
    __syncthreads();
  }
  if (lane == 0) atomic_max_u64(&T.counters[CNT_MAX_STACK], (unsigned long long)maxsp);
  const double hw = wave_max(hm);
  if (hmax) *hmax = hw;
  if (harg) *harg = wave_min_u(hm == hw ? ha : 0xFFFFFFFFu);
  if (nlum) *nlum = lum;
  return cnt;
}

// Opening criterion (Section 2.5.2): open if the cell reaches into the p-p
// sphere or B/d > theta (d to the nearest point of the cell, B from the
// luminosity centre to the farthest corner), compared as squares.
__device__ inline bool open_cell(const double lo[3], const double hi[3], const double cn[3],
                                 const double c[3], double r2, double theta2) {
  const double d2 = dist2_box(lo, hi, c);
  double e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = cn[a] - lo[a], w = hi[a] - cn[a];
    e[a] = fmax(u * u, w * w);
  }
  const double B2 = e[0] + e[1] + e[2];
  return (d2 < r2) || (B2 > theta2 * d2);
}

__device__ inline uint32_t source_pixel(int nside, double vx, double vy, double vz) {
  if (vx == 0.0 && vy == 0.0 && vz == 0.0) return 0u;
  return (uint32_t)healpix_pixel(nside, vx, vy, vz);
}


// ------------------------------------------------- element intensity kernel
// Shape f(x) of the element-averaged intensity, x = r/(R h), R = (3/4pi)^(1/2)
// (Section 2.2, eq. intint): 1 + (1-x^2) atanh(x)/x below 1, 1 - (x^2-1)
// atanh(1/x)/x above, and for x >= 2 the series sum 2 x^-2k/(4k^2-1).
__device__ inline float fshape(float x) {
  if (x < 1.0f) {
    if (x == 0.0f) return 2.0f;
    const float at = 0.5f * log1pf(2.0f * x / (1.0f - x));
    return 1.0f + (1.0f - x) * (1.0f + x) * at / x;
  }
  if (x < 2.0f) {
    if (x == 1.0f) return 1.0f;
    const float at = 0.5f * logf((x + 1.0f) / (x - 1.0f));
    return 1.0f - (x - 1.0f) * (x + 1.0f) * at / x;
  }
  const float y2 = __builtin_amdgcn_rcpf(x * x);
  float s = 2.0f / 483.0f;
  s = __builtin_fmaf(s, y2, 2.0f / 399.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 323.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 255.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 195.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 143.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 99.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 63.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 35.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 15.0f);
  s = __builtin_fmaf(s, y2, 2.0f / 3.0f);
  return s * y2;
}


struct RecvInfo {
  double x[3];
  double h;
  float rel[3];    // position relative to the bucket centre
  float inv_rh;    // 1/(R h)
  float kfac;      // 1/(2 h^2)
  uint32_t slot;
};

// ------------------------------------------------------------ near field
// Particle-particle transfer inside the p-p sphere (Section 2.4), in two
// kernels of 256 threads per bucket that stage the p-p set through LDS
// kNChunk elements at a time.  Elements are culled kSub (or kSub / 2, a
// launch option) at a time with FP32 boxes (each element's position grown by
// its own size h, plus a margin),
// which is conservative: an element can only absorb on a line that passes
// within h of it.  Threads are mapped receiver-fastest, so the lines of a
// wavefront are nearly parallel and skip the same boxes.
constexpr int kSub = 16;
constexpr int kNSub = kNChunk / kSub;

// Queue of exact-test jobs per wavefront (element-major p-p passes), one
// job per (element, source run): room for the 63 a batch of 64 leaves plus
// the largest enqueue (one per lane).
constexpr uint32_t kJobQ = 128;
// p-p sets from this size on are swept element-major by the p-p source kernel
// (each element against the pass's source runs, exact tests queued), and so
// are smaller ones whose pairs all fit one pass; the rest pair-major over
// culling boxes of staged elements.  Measured (forward p-p sources): from
// 4096 to 256 with the one-pass rule, clumpy 2^18 3.43 -> 2.66 ms, batched
// 590 -> 573 ms, the 2^21 diffuse scene (every element emits, so many
// passes over small sets) unchanged; below 256 the diffuse scene slows by
// a third.
constexpr uint32_t kPpElementMajor = 256;

// ---------------------------------------------------------- p-p job log
// The forward's element-major p-p source sweep can keep for the adjoint the
// jobs that passed its culling tests, so that the adjoint runs only the
// exact tests (the decisions are the same on both sides: the same tests on
// the same values).  Each wavefront writes one stream of 16-bit entries:
// per pass, the number of its chunks of kNT p-p elements that have jobs of
// the wavefront, then per such chunk a record -- the chunks skipped since
// the previous record and the number of jobs, two entries in one block --
// followed by the jobs (element lane << 8 | first pair of the source run).
// A stream lives in blocks of kLogBlock entries taken from a device counter
// as it grows; the last two entries of a block hold the index of the
// stream's next block.  tab[4 bucket + wave] is where a bucket's stream
// starts (block, entry); block kLogNone in tab[4 bucket] marks a bucket the
// log does not cover (a pair-major receiver chunk, or no block left), which
// the adjoint culls again itself.
constexpr uint32_t kLogBlock = 1u << 14;
constexpr uint32_t kLogData = kLogBlock - 2;   // entries per block before the link
constexpr uint32_t kLogNone = 0xFFFFFFFFu;     // no block: the stream is dead
constexpr uint32_t kLogFresh = 0xFFFFFFFEu;    // no block taken yet
constexpr uint32_t kLogMaxNear = 1u << 24;     // larger p-p sets are not logged

struct JobLog {
  uint16_t* log;       // blocks * kLogBlock entries (null: no log)
  uint2* tab;          // [bucket][4] stream starts
  uint32_t* next;      // blocks taken (zeroed before the forward)
  uint32_t blocks;
};

// A wavefront's place in its stream (wave-uniform).
struct LogPos {
  uint32_t blk, pos;
};

// A new block for the stream (kLogNone when none is left); the whole
// wavefront calls it.
__device__ inline uint32_t log_take_block(const JobLog& J) {
  uint32_t b = 0;
  if ((threadIdx.x & 63) == 0) b = atomicAdd(J.next, 1u);
  b = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)b, 0));
  return b < J.blocks ? b : kLogNone;
}

// Makes the stream writable at p (takes its first block); false if dead.
__device__ inline bool log_ready(const JobLog& J, LogPos& p) {
  if (p.blk == kLogFresh) {
    p.blk = log_take_block(J);
    p.pos = 0;
  }
  return p.blk != kLogNone;
}

// Appends cnt <= 64 entries (wave-uniform): entry k is v of the lane that
// has it (mine).  Returns the index in the log of entry 0 (for a later
// rewrite), or ~0 when the stream is dead.
__device__ inline size_t log_put(const JobLog& J, LogPos& p, uint32_t cnt, bool mine, uint32_t k,
                                 uint16_t v) {
  if (!log_ready(J, p)) return ~(size_t)0;
  uint32_t nb = p.blk;
  if (p.pos + cnt > kLogData) {
    nb = log_take_block(J);
    if ((threadIdx.x & 63) == 0) {
      J.log[(size_t)p.blk * kLogBlock + kLogData] = (uint16_t)(nb & 0xFFFFu);
      J.log[(size_t)p.blk * kLogBlock + kLogData + 1] = (uint16_t)(nb >> 16);
    }
  }
  const size_t first = p.pos < kLogData ? (size_t)p.blk * kLogBlock + p.pos
                       : nb != kLogNone ? (size_t)nb * kLogBlock : ~(size_t)0;
  if (mine) {
    const uint32_t e = p.pos + k;
    if (e < kLogData) J.log[(size_t)p.blk * kLogBlock + e] = v;
    else if (nb != kLogNone) J.log[(size_t)nb * kLogBlock + (e - kLogData)] = v;
  }
  if (p.pos + cnt > kLogData) {
    p.pos = p.pos + cnt - kLogData;
    p.blk = nb;
  } else {
    p.pos += cnt;
  }
  return first;
}

// Reserves two entries of one block (a record, written later; writer and
// reader skip the last data entry of a block when only it is left): the
// index in the log of the first, or ~0 when the stream is dead.
__device__ inline size_t log_record(const JobLog& J, LogPos& p) {
  if (!log_ready(J, p)) return ~(size_t)0;
  if (p.pos + 2 > kLogData) {
    const uint32_t nb = log_take_block(J);
    if ((threadIdx.x & 63) == 0) {
      J.log[(size_t)p.blk * kLogBlock + kLogData] = (uint16_t)(nb & 0xFFFFu);
      J.log[(size_t)p.blk * kLogBlock + kLogData + 1] = (uint16_t)(nb >> 16);
    }
    p.blk = nb;
    p.pos = 0;
    if (nb == kLogNone) return ~(size_t)0;
  }
  const size_t first = (size_t)p.blk * kLogBlock + p.pos;
  p.pos += 2;
  return first;
}

// The stream's next block after p.blk (the link the writer left), kept in
// range.
__device__ inline uint32_t log_link(const JobLog& J, uint32_t blk) {
  const uint32_t b = (uint32_t)J.log[(size_t)blk * kLogBlock + kLogData] |
                     ((uint32_t)J.log[(size_t)blk * kLogBlock + kLogData + 1] << 16);
  return b < J.blocks ? b : 0u;
}

// Reads cnt <= 64 entries (wave-uniform): lane k < cnt gets entry k.
__device__ inline uint32_t log_get(const JobLog& J, LogPos& p, uint32_t cnt, uint32_t k) {
  const uint32_t nb = p.pos + cnt > kLogData ? log_link(J, p.blk) : p.blk;
  uint32_t v = 0;
  if (k < cnt) {
    const uint32_t e = p.pos + k;
    v = e < kLogData ? J.log[(size_t)p.blk * kLogBlock + e]
                     : J.log[(size_t)nb * kLogBlock + (e - kLogData)];
  }
  if (p.pos + cnt > kLogData) {
    p.pos = p.pos + cnt - kLogData;
    p.blk = nb;
  } else {
    p.pos += cnt;
  }
  return v;
}

// Reads a record (see log_record): lane 0 gets its first entry, lane 1 its
// second.
__device__ inline uint32_t log_get_record(const JobLog& J, LogPos& p, uint32_t k) {
  if (p.pos + 2 > kLogData) {
    p.blk = log_link(J, p.blk);
    p.pos = 0;
  }
  const uint32_t v = k < 2u ? J.log[(size_t)p.blk * kLogBlock + p.pos + k] : 0u;
  p.pos += 2;
  return v;
}

// Skips cnt entries (wave-uniform).
__device__ inline void log_skip(const JobLog& J, LogPos& p, uint32_t cnt) {
  while (p.pos + cnt > kLogData) {
    cnt -= kLogData - p.pos;
    p.blk = log_link(J, p.blk);
    p.pos = 0;
  }
  p.pos += cnt;
}


// Per source run of an element-major p-p sweep (LDS, one entry per pair,
// read at the run's first pair): s = jr the source relative to the bucket
// centre, jinv = 1/|s|^2, lim = |s| + the receivers' reach R (a 1e-5
// margin), and the round cone's k2 = 1 - R^2/|s|^2 and m2 = R^2 / (|s|^2
// (|s|^2 - R^2)), m2 < 0 when |s| <= R.
struct RunTab {
  const float (*jr)[3];
  const float *jinv, *lim, *k2, *m2;
};

__device__ inline void run_tab_entry(const float s[3], float reach, float (*jr)[3], float* jinv,
                                     float* lim, float* k2, float* m2, int t) {
  const float L2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
  const float R = reach * (1.0f + 1e-5f), R2 = R * R;
  jr[t][0] = s[0];
  jr[t][1] = s[1];
  jr[t][2] = s[2];
  jinv[t] = L2 > 0.0f ? 1.0f / L2 : 0.0f;
  lim[t] = (cull_sqrt(L2) + reach) * (1.0f + 1e-5f);
  k2[t] = L2 > R2 ? (L2 - R2) / L2 : 0.0f;
  m2[t] = L2 > R2 ? R2 / (L2 * (L2 - R2)) : -1.0f;
}

// Whether p comes within A - R u of the point u s of the segment from the
// origin to s, for some u in [0, 1]: the round cone swept by spheres shrinking
// from radius A at the origin to A - R at s.  Every segment from a point
// within R of the origin to s lies inside the cone of radius R (1 - u)
// around u s, so an element of size h can touch one only if it passes with
// A = h + R.  min over u of |p - u s| + R u is convex; its free minimum is
// at u* = t0 - d m (t0 the projection parameter, d the distance to the
// line, m = R / (|s| sqrt(|s|^2 - R^2))) with value d sqrt(1 - R^2/|s|^2)
// + R t0, else at an end (u = 0: |p|, u = 1: |p - s| + R); when |s| <= R it
// is at u = 0.  All in squares (no square roots); A is widened by 1e-4
// relative plus tol for FP32 rounding.
__device__ inline bool round_cone(const float p[3], const float s[3], float jinv, float k2, float m2,
                                  float R, float A, float tol) {
#pragma clang fp contract(fast)   // FP32 culling with margins: fused products are fine
  const float Ap = A * (1.0f + 1e-4f) + tol;
  const float pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const float f0 = p[0] - s[0], f1 = p[1] - s[1], f2 = p[2] - s[2];
  const float fs = f0 * f0 + f1 * f1 + f2 * f2;
  const float t0 = (p[0] * s[0] + p[1] * s[1] + p[2] * s[2]) * jinv;
  const float d0 = p[0] - t0 * s[0], d1 = p[1] - t0 * s[1], d2 = p[2] - t0 * s[2];
  const float dp2 = d0 * d0 + d1 * d1 + d2 * d2;
  const float dm = dp2 * m2;
  const bool lo = m2 < 0.0f || t0 < 0.0f || t0 * t0 < dm;
  const bool hi = t0 > 1.0f && (t0 - 1.0f) * (t0 - 1.0f) > dm;
  const float B = Ap - R, e = Ap - R * t0;
  const bool at0 = pp <= Ap * Ap;
  const bool at1 = B >= 0.0f && fs <= B * B;
  const bool mid = e >= 0.0f && dp2 * k2 <= e * e;
  return lo ? at0 : (hi ? at1 : mid);
}

// The p-p elements of a wavefront in an element-major sweep (one per lane
// with `has`, positions pr relative to the bucket centre, each with its
// size hrad, margins included) as one sphere per quarter-wavefront (16
// lanes), written to G[4][5]: centre g = G[q][0..2] (the middle of their
// box), G[q][3] = rp the farthest position from g, G[q][4] = rr the
// farthest position plus its size (< 0 when no lane of the quarter holds an
// element).  The elements of a slot-ordered p-p list are spatially close in
// runs of 16, so most source runs miss a quarter's sphere and skip its
// per-element tests.
constexpr int kElemGroup = 16;
// Minimum / maximum over each group of 16 lanes, in every lane of the group,
// by DPP moves (swap neighbours, swap pairs, mirror half rows, mirror rows).
// Call with every lane active.
__device__ inline float dpp_mov(float v, int ctrl) {
  switch (ctrl) {
    case 0: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
    case 1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
    case 2: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));
    default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));
  }
}
__device__ inline float quarter_fmin(float v) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v = fminf(v, dpp_mov(v, k));
  return v;
}
__device__ inline float quarter_fmax(float v) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v = fmaxf(v, dpp_mov(v, k));
  return v;
}
__device__ inline void elem_group(const float pr[3], float hrad, bool has, float (*G)[5]) {
  float g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    g[a] = 0.5f * (quarter_fmin(has ? pr[a] : INFINITY) + quarter_fmax(has ? pr[a] : -INFINITY));
  const float d0 = pr[0] - g[0], d1 = pr[1] - g[1], d2 = pr[2] - g[2];
  const float dl = cull_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const float rp = quarter_fmax(has ? dl : -1.0f);
  const float rr = quarter_fmax(has ? dl + hrad : -1.0f);
  const int lane = (int)(threadIdx.x & 63);
  if ((lane & (kElemGroup - 1)) == 0) {
    float* q = G[lane / kElemGroup];
    q[0] = g[0];
    q[1] = g[1];
    q[2] = g[2];
    q[3] = rp;
    q[4] = rr;
  }
  wave_lds_sync();
}

// The (quarter, source run) pairs, bit 16 quarter + k for run k0 + k (k <
// 16; lane 16 quarter + k tests it; pair (k0 + k) * nrecv), for which some
// element of the quarter can pass the per-element test: the sphere's centre
// within the round cone of radius rr + R(1 - u) (R the reach, with its
// margin) and within lim + rp of the source.  Margins of 1e-4
// relative and 1e-5 of the coordinates' size cover FP32 rounding on both
// sides.  Wave-uniform mask.
__device__ inline uint64_t group_runs(const float (*G)[5], const RunTab& RT, float R, int k0,
                                      int nruns, int nrecv) {
#pragma clang fp contract(fast)   // FP32 culling with margins: fused products are fine
  const int lane = (int)(threadIdx.x & 63);
  const float* Gq = G[lane / kElemGroup];
  const int k = k0 + (lane & (kElemGroup - 1));
  const float rr = Gq[4];
  bool pass = false;
  if (k < nruns && rr >= 0.0f) {
    const float g[3] = {Gq[0], Gq[1], Gq[2]};
    const float rp = Gq[3];
    const int q = k * nrecv;
    const float s[3] = {RT.jr[q][0], RT.jr[q][1], RT.jr[q][2]};
    const float tol = 1e-5f * (fabsf(g[0]) + fabsf(g[1]) + fabsf(g[2]) + fabsf(s[0]) +
                               fabsf(s[1]) + fabsf(s[2]));
    const float f0 = g[0] - s[0], f1 = g[1] - s[1], f2 = g[2] - s[2];
    const float r2 = (RT.lim[q] + rp) * (1.0f + 1e-4f) + tol;
    pass = (f0 * f0 + f1 * f1 + f2 * f2 <= r2 * r2) &
           round_cone(g, s, RT.jinv[q], RT.k2[q], RT.m2[q], R, rr * (1.0f + 1e-4f) + R, tol);
  }
  return ballot64(pass);
}

// Takes up to four set bits from the wave-uniform mask *gm (lowest first)
// and gives lane 16 i + j the i-th of them (-1 past the last): the (quarter,
// run) pair whose element j that lane tests.
__device__ inline int take_quarter_pair(uint64_t* gm) {
  uint64_t m = *gm;
  int b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    b[i] = m ? (int)__builtin_ctzll(m) : -1;
    m &= m - 1ull;
  }
  *gm = m;
  const int i = (int)(threadIdx.x & 63) / kElemGroup;
  const int r01 = (i & 1) ? b[1] : b[0], r23 = (i & 1) ? b[3] : b[2];
  return (i & 2) ? r23 : r01;
}

// The per-element test of an element-major sweep against source run q (its
// first pair): no farther from the source than lim, and within hrad
// + R of the centre's segment to the source (the cylinder around the round
// cone, cheaper to test); a superset of the elements the exact test finds
// on any of the run's pairs.  A NaN hrad (a lane without an element) fails.
__device__ inline bool elem_run_test(const float pr[3], float hrad, const RunTab& RT, float R,
                                     int q) {
#pragma clang fp contract(fast)   // FP32 culling with margins: fused products are fine
  const float s0 = RT.jr[q][0], s1 = RT.jr[q][1], s2 = RT.jr[q][2];
  const float f0 = pr[0] - s0, f1 = pr[1] - s1, f2 = pr[2] - s2;
  float tt = (pr[0] * s0 + pr[1] * s1 + pr[2] * s2) * RT.jinv[q];
  tt = fminf(1.0f, fmaxf(0.0f, tt));
  const float d0 = pr[0] - tt * s0, d1 = pr[1] - tt * s1, d2 = pr[2] - tt * s2;
  const float rad = hrad + R, lim = RT.lim[q];
  // both conditions evaluated (no branch between their LDS reads)
  return (f0 * f0 + f1 * f1 + f2 * f2 <= lim * lim * (1.0f + 1e-4f)) &
         (d0 * d0 + d1 * d1 + d2 * d2 <= rad * rad);
}

// The queued (element, source run) jobs that also pass the round cone
// (elements within hrad + R (1 - u) of the centre's segment): the filter
// between the per-element test and the exact tests.
__device__ inline bool elem_run_cone(const float pr[3], float hrad, const RunTab& RT, float R,
                                     int q) {
#pragma clang fp contract(fast)   // FP32 culling with margins: fused products are fine
  const float s[3] = {RT.jr[q][0], RT.jr[q][1], RT.jr[q][2]};
  const float tol = 1e-5f * (fabsf(pr[0]) + fabsf(pr[1]) + fabsf(pr[2]) + fabsf(s[0]) +
                             fabsf(s[1]) + fabsf(s[2]));
  return round_cone(pr, s, RT.jinv[q], RT.k2[q], RT.m2[q], R, hrad + R, tol);
}

template <int NB> struct NearTile {
  double x[kNChunk], y[kNChunk], z[kNChunk], h2[kNChunk];
  float sig[kNChunk], invh[kNChunk];
  float kap[kNChunk][NB];
  uint32_t slot[kNChunk];
  float blo[kNSub][3], bhi[kNSub][3];              // per kSub elements
  float blo8[2 * kNSub][3], bhi8[2 * kNSub][3];    // per kSub / 2 elements
};

// Culling boxes of a staged chunk at the granularity `sub` (kSub or kSub / 2).
template <int NB>
__device__ inline const float (*near_boxes(const NearTile<NB>& S, int sub, bool hi))[3] {
  if (sub == kSub) return hi ? S.bhi : S.blo;
  return hi ? S.bhi8 : S.blo8;
}

// Sum over each group of `sub` (16 or 8) consecutive lanes, returned in every
// lane of the group, by DPP moves (swap neighbours, swap pairs, mirror half
// rows, mirror rows).  Call with every lane active.
__device__ inline float group_sum_dpp(float v, int sub) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));
  if (sub == 16)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));
  return v;
}

template <int NB>
__device__ inline void stage_near(NearTile<NB>& S, const DevTree& T, const uint32_t* near,
                                  uint32_t c0, uint32_t cl, const double c[3]) {
  const int t = threadIdx.x;
  __syncthreads();
  if ((uint32_t)t < cl) {
    const uint32_t l = near[c0 + t];
    const double hl = T.h[l];
    S.x[t] = (double)T.x[l];
    S.y[t] = (double)T.y[l];
    S.z[t] = (double)T.z[l];
    S.h2[t] = hl * hl;
    const float iv = __builtin_amdgcn_rcpf((float)hl);   // values, not decisions: FP32
    S.invh[t] = iv;
    S.sig[t] = (float)(3.0 / kPi) * T.m[l] * iv * iv;
#pragma unroll
    for (int b = 0; b < NB; ++b) S.kap[t][b] = T.kappa[(int64_t)b * T.n + l];
    S.slot[t] = l;
  }
  __syncthreads();
  if (t < 2 * kNSub) {
    constexpr int kHalf = kSub / 2;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int u1 = min((int)cl, (t + 1) * kHalf);
    for (int u = t * kHalf; u < u1; ++u) {
      const float h = cull_sqrt((float)S.h2[u]);
      const float p[3] = {(float)(S.x[u] - c[0]), (float)(S.y[u] - c[1]), (float)(S.z[u] - c[2])};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float m = h + 1e-5f * (fabsf(p[a]) + h);
        lo[a] = fminf(lo[a], p[a] - m);
        hi[a] = fmaxf(hi[a], p[a] + m);
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) { S.blo8[t][a] = lo[a]; S.bhi8[t][a] = hi[a]; }
  }
  __syncthreads();
  if (t < kNSub) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.blo[t][a] = fminf(S.blo8[2 * t][a], S.blo8[2 * t + 1][a]);
      S.bhi[t][a] = fmaxf(S.bhi8[2 * t][a], S.bhi8[2 * t + 1][a]);
    }
  }
  __syncthreads();
}

// Next chunk of active bucket members: the first kRMax active ones from the
// cursor, in member order.  Wavefront 0 tests 64 members at a time (its lanes
// keep the cursor, identical in each).
__device__ inline int load_receivers(const DevTree& T, const uint8_t* active, const double c[3],
                                     uint32_t& member, uint32_t mend, RecvInfo* recv,
                                     uint32_t* nrecv_s) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t k = 0;
    while (member < mend && k < (uint32_t)kRMax) {
      const uint32_t s = member + (uint32_t)lane;
      const bool act = s < mend && (active == nullptr || active[T.perm[s]]);
      const uint64_t m = ballot64(act);
      const uint32_t pos = k + (uint32_t)mbcnt(m);
      if (act && pos < (uint32_t)kRMax) {
        RecvInfo ri;
        ri.x[0] = (double)T.x[s];
        ri.x[1] = (double)T.y[s];
        ri.x[2] = (double)T.z[s];
        ri.h = T.h[s];
        for (int a = 0; a < 3; ++a) ri.rel[a] = (float)(ri.x[a] - c[a]);
        ri.inv_rh = (float)(1.0 / (kR * ri.h));
        ri.kfac = (float)(1.0 / (2.0 * ri.h * ri.h));
        ri.slot = s;
        recv[pos] = ri;
      }
      const uint32_t cnt = (uint32_t)__popcll(m);
      if (k + cnt > (uint32_t)kRMax) {   // resume at the first active member not taken
        uint64_t rest = m;
        for (uint32_t j = k; j < (uint32_t)kRMax; ++j) rest &= rest - 1ull;
        member += (uint32_t)(__ffsll((long long)rest) - 1);
        k = (uint32_t)kRMax;
      } else {
        k += cnt;
        member = min(member + 64u, mend);
      }
    }
    if (lane == 0) *nrecv_s = k;
  }
  __syncthreads();
  return (int)*nrecv_s;
}

// FP32 ray-box test on the half line o + t n, t >= 0 (inv = 1/n, +-huge for 0).
__device__ inline bool ray_meets_box(const float o[3], const float inv[3], const float lo[3],
                                     const float hi[3]) {
  float tin = 0.0f, tout = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t1 = (lo[a] - o[a]) * inv[a], t2 = (hi[a] - o[a]) * inv[a];
    tin = fmaxf(tin, fminf(t1, t2));
    tout = fminf(tout, fmaxf(t1, t2));
  }
  return tin <= tout;
}

// ------------------------------------------------------------- far field
constexpr int kFT = 256;   // threads of the far-field kernels

// Sources of a (bucket, ray group) whose cell optical depths the forward
// keeps for the adjoint when all of them fit one window of both kernels.
template <int NB> struct KeptCap {
  static constexpr int value = NB == 1 ? 512 : NB <= 3 ? 448 : NB == 4 ? 192 : NB == 6 ? 224
                               : 256;
};
// Sources per LDS window of the forward far-field kernel: as many as let
// four workgroups share a CU's 160 KiB of LDS up to five bands (three at
// six, two from seven bands on, where registers limit it anyway).
template <int NB> struct SrcCap {
  static constexpr int value = NB <= 2 ? 512 : NB == 3 ? 448 : NB == 4 ? 320 : NB == 6 ? 224 : 256;
};

// Block-wide compaction: position of this thread's item among the set ones
// (in thread order) and the block total.  Uses wcnt[4] in LDS; two barriers.
__device__ inline uint32_t block_compact(bool pred, uint32_t* wcnt, uint32_t* total) {
  const int t = threadIdx.x, wv = t >> 6;
  const uint64_t m = ballot64(pred);
  if ((t & 63) == 0) wcnt[wv] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kFT / 64; ++w) {
    if (w < wv) base += wcnt[w];
    tot += wcnt[w];
  }
  __syncthreads();
  *total = tot;
  return base + (uint32_t)mbcnt(m);
}

// Directions of one group of up to 64 rays: FP64 (exact ray-box tests),
// their reciprocals and an FP32 copy (conservative candidate filter).
// The rays that can meet a p-p element from a receiver (d = the element's
// offset from the receiver, dd = |d|^2, h2 = its size squared): a ray meets
// it (ahead, b < h) only if its direction lies within asin(h/|d|) of d, so
// its z (cos of the polar angle) lies within the z-range of that cone.  The
// HEALPix ring order lists the rays by decreasing z, ring by ring (ring i of
// 4N - 1 at z = 1 - i^2/(3N^2) in the north cap, 4/3 - 2i/(3N) in the belt),
// so those rays are one index range [*ka, *kb): the rings inside the cone's
// z-range, widened by 1e-4 in sin and z and 1e-3 of a ring for FP32
// rounding.  The receiver inside the element (h near |d|): every ray.
__device__ inline float ring_of_z(int N, float z) {
  if (z > 2.0f / 3.0f) return (float)N * cull_sqrt(3.0f * fmaxf(1.0f - z, 0.0f));
  if (z < -2.0f / 3.0f) return 4.0f * N - (float)N * cull_sqrt(3.0f * fmaxf(1.0f + z, 0.0f));
  return 2.0f * N - 1.5f * N * z;
}
__device__ inline int ring_start(int N, int i) {
  if (i <= N) return 2 * i * (i - 1);
  if (i <= 3 * N) return 2 * N * (N - 1) + 4 * N * (i - N);
  const int ii = 4 * N - i + 1;   // rings from i to the south pole: ii
  return 12 * N * N - 2 * ii * (ii - 1);
}
__device__ inline void ray_ring_range(int N, double d0, double d1, double d2, double dd, double h2,
                                      int* ka, int* kb) {
  const float ddf = (float)dd;
  const float s2 = (float)h2 / ddf;
  if (!(s2 < 0.99f)) {
    *ka = 0;
    *kb = 12 * N * N;
    return;
  }
  const float z = (float)d2 * rsqrtf(ddf);
  const float sa = fminf(cull_sqrt(s2) * (1.0f + 1e-4f) + 1e-4f, 1.0f);
  const float ca = cull_sqrt(fmaxf(1.0f - sa * sa, 0.0f));
  const float st = cull_sqrt(fmaxf(1.0f - z * z, 0.0f));
  const float zhi = (z >= ca) ? 1.0f : fminf(z * ca + st * sa + 1e-4f, 1.0f);
  const float zlo = (-z >= ca) ? -1.0f : fmaxf(z * ca - st * sa - 1e-4f, -1.0f);
  const int i0 = max(1, (int)ceilf(ring_of_z(N, zhi) - 1e-3f));
  const int i1 = min(4 * N - 1, (int)floorf(ring_of_z(N, zlo) + 1e-3f));
  if (i0 > i1) {
    *ka = *kb = 0;
    return;
  }
  *ka = ring_start(N, i0);
  *kb = ring_start(N, i1 + 1);
}

// Rays per group of the p-p column kernels.  Their pair loop computes each
// (p-p element, receiver) pair's ring range and loads its element once per
// group, so a group holds every ray up to N_side 4 where the LDS sums of a
// group allow it (up to four bands); the candidate masks stay 64 rays wide.
template <int NB> struct PpRayGroup {
  static constexpr int value = NB <= 4 ? 192 : 64;
};

struct RayGroup {
  double n[64][3], inv[64][3];
  float nf[64][3];
  int cls[64];   // direction class (transmission tables)
};

// The directed ray of the bucket centred at c (TREVR_DIRECTED) takes its
// aimed direction; its class stays that of its HEALPix direction.
__device__ inline void load_ray_group(const DevTree& T, const double c[3], int k0, int kn,
                                      RayGroup& G) {
  const int t = threadIdx.x;
  if (t < kn) {
    const int k = k0 + t;
    double u[3];
    const int kd = directed_ray(T, c, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double na = (k == kd) ? u[a] : T.ray_n[3 * k + a];
      G.n[t][a] = na;
      G.inv[t][a] = (na != 0.0) ? 1.0 / na : 0.0;
      G.nf[t][a] = (float)na;
    }
    G.cls[t] = T.ray_class[k];
  }
}

// Far sources of a ray group held in LDS, CAP at a time: position relative
// to the bucket centre, distance s projected on the ray of their pixel (the
// end of the cell trace: with the complex source model, s less the length
// of the source's own ray),
// per-band luminosity, accumulated cell optical depth (tau, plus suffix
// adds in sfx unless the user keeps those elsewhere), the ray (in the group)
// and the per-ray order by s.
template <int CAP, int NB, bool kSfx = true> struct SrcWindow {
  float rel[CAP][3];
  float s[CAP];
  float tau[CAP][NB];
  float sfx[kSfx ? CAP : 1][NB];
  float L[CAP][NB];
  uint8_t ray[CAP];
  uint16_t order[CAP];
  uint32_t ray_beg[65], ray_fill[64];
};

// Cut-list source id as kept by the adjoint: element slot, or node with
// this bit set for merged cell sources.
constexpr uint32_t kSrcCellBit = 0x80000000u;

// Stage the sources whose pixel lies in rays [k0, k0 + kn), taking those
// with group index in [skip, skip + CAP) (group index = order in the cut
// list).  Returns the number of sources of the group.  `ids` (optional)
// receives each staged source's id.
template <int CAP, int NB, bool kSfx>
__device__ inline uint32_t stage_window(const DevTree& T, const uint2* mycut, uint32_t ncut,
                                        const double c[3], int k0, int kn, uint32_t skip,
                                        SrcWindow<CAP, NB, kSfx>& W, uint32_t* wcnt,
                                        uint32_t* ids) {
  const int t = threadIdx.x;
  const int64_t n = T.n;
  uint32_t nsg_all = 0;
  for (uint32_t e0 = 0; e0 < ncut; e0 += kFT) {
    const uint32_t e = e0 + (uint32_t)t;
    bool mine = false;
    uint2 ent = make_uint2(0, 0);
    uint32_t pix = CUT_NOPIX;
    if (e < ncut) {
      ent = mycut[e];
      pix = ent.y & 0xFFFFu;
      mine = pix != CUT_NOPIX && (int)pix >= k0 && (int)pix < k0 + kn;
    }
    uint32_t tot;
    const uint32_t gi = nsg_all + block_compact(mine, wcnt, &tot);
    if (mine && gi >= skip && gi < skip + (uint32_t)CAP) {
      const uint32_t slot = gi - skip;
      double p[3];
      float Lv[NB];
      const bool part = (ent.y & CUT_KIND_MASK) == CUT_PART;
      if (part) {
        p[0] = (double)T.x[ent.x];
        p[1] = (double)T.y[ent.x];
        p[2] = (double)T.z[ent.x];
#pragma unroll
        for (int b = 0; b < NB; ++b) Lv[b] = T.lum[(int64_t)b * n + ent.x];
      } else {
        const double4 cn = T.cen[ent.x];
        p[0] = cn.x;
        p[1] = cn.y;
        p[2] = cn.z;
#pragma unroll
        for (int b = 0; b < NB; ++b) Lv[b] = (float)T.Lb[(int64_t)ent.x * NB + b];
      }
      const double v0 = p[0] - c[0], v1 = p[1] - c[1], v2 = p[2] - c[2];
      double sd = 0.0;
      if (!(v0 == 0.0 && v1 == 0.0 && v2 == 0.0)) {
        double u[3];
        const bool dir = directed_ray(T, c, u) == (int)pix;
        const double* nn = dir ? u : &T.ray_n[3 * pix];
        sd = v0 * nn[0] + v1 * nn[1] + v2 * nn[2];
      }
      if (!part && T.csrc_d) {
        // complex source model (Section 2.7): the merged source's own ray
        // toward the receiver (emission direction -n_k, the antipodal
        // pixel) attenuates its luminosity, and the cell trace stops at the
        // projected end of that ray, the edge of the source's cell
        const int64_t row = (int64_t)ent.x * T.nray + T.ray_anti[pix];
        const double d = T.csrc_d[row];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          Lv[b] = (float)((double)Lv[b] * exp(-T.csrc_a[row * NB + b] * d));
        sd -= d;
      }
      W.rel[slot][0] = (float)v0;
      W.rel[slot][1] = (float)v1;
      W.rel[slot][2] = (float)v2;
      W.s[slot] = (float)sd;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        W.L[slot][b] = Lv[b];
        W.tau[slot][b] = 0.0f;
        if constexpr (kSfx) W.sfx[slot][b] = 0.0f;
      }
      W.ray[slot] = (uint8_t)(pix - k0);
      if (ids) ids[slot] = part ? ent.x : (ent.x | kSrcCellBit);
    }
    nsg_all += tot;
  }
  return nsg_all;
}

// Bin the staged sources by ray and order each ray's sources by s (ties by
// staging index): each source's rank among its ray's sources is counted by
// the thread holding it, O(sources on the ray) each, all threads at once.  The
// owner of a ray (threads t < 64) gets its range [q0, q1) of W.order.  Ends
// with a barrier: every thread may then read any ray's list.
template <int CAP, int NB, bool kSfx>
__device__ inline void sort_window(SrcWindow<CAP, NB, kSfx>& W, uint32_t nsg, bool rt,
                                   uint32_t& q0, uint32_t& q1) {
  constexpr int kPer = (CAP + kFT - 1) / kFT;   // sources per thread
  const int t = threadIdx.x;
  if (t < 64) W.ray_fill[t] = 0u;
  __syncthreads();
  for (uint32_t q = t; q < nsg; q += kFT) atomicAdd(&W.ray_fill[W.ray[q]], 1u);
  __syncthreads();
  if (t < 64) {
    const uint32_t v = W.ray_fill[t];
    const uint32_t ex = wave_excl(v, t);
    W.ray_beg[t] = ex;
    if (t == 63) W.ray_beg[64] = ex + v;
    W.ray_fill[t] = ex;
  }
  __syncthreads();
  for (uint32_t q = t; q < nsg; q += kFT) {
    const uint32_t pos = atomicAdd(&W.ray_fill[W.ray[q]], 1u);
    W.order[pos] = (uint16_t)q;
  }
  __syncthreads();
  uint32_t dst[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t q = (uint32_t)t + (uint32_t)k * kFT;
    dst[k] = 0xFFFFFFFFu;
    if (q < nsg) {
      const uint32_t r = W.ray[q], b0 = W.ray_beg[r], b1 = W.ray_beg[r + 1];
      const float sq = W.s[q];
      uint32_t rank = 0;
      for (uint32_t a = b0; a < b1; ++a) {
        const uint32_t o = W.order[a];
        const float so = W.s[o];
        rank += (so < sq || (so == sq && o < q)) ? 1u : 0u;
      }
      dst[k] = b0 + rank;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (dst[k] != 0xFFFFFFFFu) W.order[dst[k]] = (uint16_t)((uint32_t)t + (uint32_t)k * kFT);
  q0 = rt ? W.ray_beg[t] : 0u;
  q1 = rt ? W.ray_beg[t + 1] : 0u;
  __syncthreads();
}

// Every (absorbing cut entry, ray of the group) hit found by the thread
// holding the entry, with no barriers: threads take the cut entries in
// turn; for an absorbing one the conservative FP32 bounding-sphere test
// gives its candidate rays, the exact FP64 ray-box test keeps those that
// meet the cell beyond the p-p sphere, and the same thread calls
// on_hit(node, ray, t0, t1, clipped) with t0 = max(t_in, r), clipped =
// (t_in < r).  Hits of one ray arrive from many threads in no fixed order,
// so on_hit must update shared state atomically.
template <class F>
__device__ inline void for_each_hit_lane(const DevTree& T, const uint2* mycut, uint32_t ncut,
                                         const double c[3], double r, int kn, const RayGroup& G,
                                         F&& on_hit) {
  const uint64_t all = (kn >= 64) ? ~0ull : ((1ull << kn) - 1ull);
  for (uint32_t e = threadIdx.x; e < ncut; e += kFT) {
    const uint2 ent = mycut[e];
    if (!(ent.y & CUT_ABS)) continue;
    const uint32_t node = ent.x;
    double lo[3], hi[3];
    node_box(T.hdr, T.nk[node], lo, hi);
    float mc[3], R2 = 0.0f, D2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mc[a] = (float)(0.5 * (lo[a] + hi[a]) - c[a]);
      const float hx = (float)(0.5 * (hi[a] - lo[a]));
      R2 += hx * hx;
      D2 += mc[a] * mc[a];
    }
    const float marg = 1e-5f * D2 + 1e-30f;
    uint64_t cand = all;
    if (D2 - R2 > marg) {
      const float thr = D2 - R2 - marg;
      cand = 0ull;
      for (int kq = 0; kq < kn; ++kq) {
        const float nm = G.nf[kq][0] * mc[0] + G.nf[kq][1] * mc[1] + G.nf[kq][2] * mc[2];
        if (nm > 0.0f && nm * nm >= thr) cand |= 1ull << kq;
      }
    }
    while (cand) {
      const int kq = __ffsll((long long)cand) - 1;
      cand &= cand - 1ull;
      double tin, tout;
      if (slab(lo, hi, c, G.n[kq], G.inv[kq], tin, tout) && tout > fmax(tin, r))
        on_hit(node, kq, fmax(tin, r), tout, tin < r);
    }
  }
}

// The same hits, queued: for light callbacks (the forward's), where lanes
// with few candidate rays would otherwise wait for the busiest.  No workgroup
// barriers: threads take the cut entries in turn; for each ray of the group
// the conservative FP32 bounding-sphere test marks the thread's entry as a
// candidate, candidates are queued per wavefront in Q (kHitQ words) and run
// 64 at a time, one per lane: the exact FP64 ray-box test keeps those that
// meet the cell beyond the p-p sphere and that lane calls on_hit(node, ray,
// t0, t1, clipped) with t0 = max(t_in, r), clipped = (t_in < r).  Hits of
// one ray arrive from many lanes in no fixed order, so on_hit must update
// shared state atomically.
constexpr uint32_t kHitQ = 128;   // one batch of 64 plus one step's 64

template <class F>
__device__ inline void for_each_hit_queued(const DevTree& T, const uint2* mycut, uint32_t ncut,
                                           const double c[3], double r, int kn, const RayGroup& G,
                                           uint32_t* Q, F&& on_hit) {
  const int lane = threadIdx.x & 63;
  uint32_t head = 0, tail = 0;   // wave-uniform queue cursors
  auto run = [&](uint32_t cnt) {
    if ((uint32_t)lane < cnt) {
      const uint32_t job = Q[(head + (uint32_t)lane) & (kHitQ - 1)];
      const uint32_t e = job >> 6;
      const int kq = (int)(job & 63u);
      const uint32_t node = mycut[e].x;
      double lo[3], hi[3];
      node_box(T.hdr, T.nk[node], lo, hi);
      double tin, tout;
      if (slab(lo, hi, c, G.n[kq], G.inv[kq], tin, tout) && tout > fmax(tin, r))
        on_hit(node, kq, fmax(tin, r), tout, tin < r);
    }
  };
  const uint32_t rounds = (ncut + kFT - 1) / kFT;
  for (uint32_t rd = 0; rd < rounds; ++rd) {
    const uint32_t e = rd * kFT + threadIdx.x;
    bool live = false, every = false;
    float mc[3] = {0.0f, 0.0f, 0.0f}, thr = 0.0f;
    if (e < ncut) {
      const uint2 ent = mycut[e];
      if (ent.y & CUT_ABS) {
        live = true;
        double lo[3], hi[3];
        node_box(T.hdr, T.nk[ent.x], lo, hi);
        float R2 = 0.0f, D2 = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          mc[a] = (float)(0.5 * (lo[a] + hi[a]) - c[a]);
          const float hx = (float)(0.5 * (hi[a] - lo[a]));
          R2 += hx * hx;
          D2 += mc[a] * mc[a];
        }
        const float marg = 1e-5f * D2 + 1e-30f;
        every = !(D2 - R2 > marg);   // the centre may be inside: every ray
        thr = D2 - R2 - marg;
      }
    }
    if (ballot64(live) == 0ull) continue;
    for (int kq = 0; kq < kn; ++kq) {
      bool cand = false;
      if (live) {
        const float nm = G.nf[kq][0] * mc[0] + G.nf[kq][1] * mc[1] + G.nf[kq][2] * mc[2];
        cand = every || (nm > 0.0f && nm * nm >= thr);
      }
      const uint64_t m = ballot64(cand);
      if (m == 0ull) continue;
      if (cand) Q[(tail + (uint32_t)mbcnt(m)) & (kHitQ - 1)] = (e << 6) | (uint32_t)kq;
      tail += (uint32_t)__popcll(m);
      wave_lds_sync();
      if (tail - head >= 64u) {
        run(64u);
        head += 64u;
        wave_lds_sync();
      }
    }
  }
  if (tail > head) run(tail - head);
}

// Gradient accumulators (sorted slots / preorder nodes), FP64.
struct Grad {
  double* gL;       // [B][n]
  double* gk;       // [B][n]
  double* gh;       // [n]   d/dh (converted to rho at the end)
  double* gr;       // [n]   direct d/drho
  double* galpha;   // [node][class][B]
  double* gLb;      // [node][B]
  double* gcen;     // [node][4]: d/d centre; later (u, v) of the centre adjoint
  double* grpp;     // [bucket] d/d r_pp
  // The far field adds to galpha, gLb and gcen from every bucket, and the
  // cells near the root are shared by most buckets: workgroups add to one
  // of ka (ks) copies of galpha (of gLb, gcen), chosen by workgroup index,
  // which spreads the atomics over more addresses; the copies are summed
  // into the first before the tree pass.
  uint32_t ka, ks;      // copies (powers of two)
  int64_t na, ns, nc;   // elements per copy: of galpha; of gLb; of gcen
  // The accumulators of one scene (arrays span every scene of a forest).
  __device__ Grad at(const DevTree& T) const {
    Grad g = *this;
    g.gL += T.joff;
    g.gk += T.joff;
    g.gh += T.eoff;
    g.gr += T.eoff;
    g.galpha += T.aoff;
    g.gLb += T.lboff;
    g.gcen += 4 * T.noff;
    return g;
  }
};

// Inputs and outputs of the adjoint's per-bucket kernels.
struct BwdArgs {
  const uint8_t* active;
  const float* bg;
  const double* gJ;
  Grad G;
  double* jraw;        // raw J per (receiver, band)
  float* gtpp;         // adjoint of the p-p columns, laid out like them
  const float* kept_tau;
  const float* kept_tex;
};

}  // namespace trevr
