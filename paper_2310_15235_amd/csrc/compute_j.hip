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
//   k_pp_rays         256 threads per bucket stage the p-p set through LDS:
//                     per receiver and ray the p-p optical depth (kept for the
//                     far field);
//   k_pp_src          the attenuated p-p sources (J starts with these);
//   k_far             one wavefront reduces the cut ray by ray: rays in groups
//                     of 64 with one lane per ray, so a lane owns its ray's
//                     sources and adds the optical depth of every absorbing
//                     cell its ray crosses without atomics; then the lanes
//                     sweep the sources against every receiver (FP64 sums),
//                     add the background and apply the thick-element factor.
// Decisions (opening test, p-p membership, the side of a receiver an element
// lies on, pixel of a source, ray-box intersection) are made in FP64 with the
// same correctly rounded operation sequence as their definition, so they are
// reproducible; transcendental physics (exp, the intensity kernel) runs in
// FP32 with FP64 accumulation.

#include <algorithm>
#include <cmath>

#include "trevr_internal.hpp"

namespace trevr {

constexpr int kRMax = 8;         // receivers per pass
constexpr int kStackCap = 4096;  // traversal stack entries (LDS)
constexpr uint32_t kCutCap = 2048;
constexpr uint32_t kBatch = 65536;   // buckets per launch (bounds the cut-list scratch)
constexpr int kCostBins = 48;
constexpr int kNT = 256;         // threads of the near-field kernel
constexpr int kNChunk = 256;     // p-p elements staged per pass
constexpr int kNPair = 2;        // (receiver, p-p source) pairs per thread per pass
constexpr int kRayPer = 2;       // rays per thread in the p-p column pass
constexpr double kR = 0.48860251190291992;   // (3/(4 pi))^(1/2)

__device__ inline void atomic_max_u64(unsigned long long* a, unsigned long long v) {
  atomicMax(a, v);
}

// ------------------------------------------------------ active buckets
__global__ void k_active_buckets(DevTree T, const uint8_t* active, uint32_t* blist,
                                 uint32_t* bnact, uint32_t* nb) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= T.num_nodes) return;
  const uint4 nk = T.nk[p];
  if (!(nk.w & META_LEAF)) return;
  const uint2 lk = T.nlink[p];
  uint32_t cnt = 0;
  for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) cnt += (active == nullptr || active[T.perm[s]]) ? 1u : 0u;
  if (cnt == 0) return;
  const uint32_t b = atomicAdd(nb, 1u);
  blist[b] = (uint32_t)p;
  bnact[b] = cnt;
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
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
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

// Range query by one wavefront: elements strictly within sqrt(r2) of c.
// Returns the count; *hmax gets their largest size, *nlum the number that
// emit.  With `out`, writes their sorted slots: luminous ones from out[0],
// the others from out[lum_total].  Boxes are pruned conservatively (an
// element can sit an ulp outside its box after quantisation); membership is
// the exact test.  The traversal stack lives in `stack` (kStackCap words).
__device__ uint32_t wave_near(const DevTree& T, const double c[3], double r2, uint32_t* stack,
                              double* hmax, uint32_t* nlum, uint32_t* out, uint32_t lum_total,
                              bool* overflow) {
  const int lane = threadIdx.x & 63;
  const double prune = r2 * (1.0 + 1e-9);
  uint32_t cnt = 0, lum = 0;
  double hm = 0.0;
  int sp = 1;
  if (lane == 0) stack[0] = 0u;
  __syncthreads();
  while (sp > 0) {
    const int take = min(sp, 64);
    sp -= take;
    const bool valid = lane < take;
    const uint32_t node = valid ? stack[sp + lane] : 0u;
    __syncthreads();
    bool push = false;
    uint32_t mine = 0, mylum = 0;
    uint2 lk = make_uint2(0, 0);
    bool isleaf = false;
    if (valid) {
      const uint4 nk = T.nk[node];
      double lo[3], hi[3];
      node_box(T.hdr, nk, lo, hi);
      if (!(dist2_box(lo, hi, c) > prune)) {
        isleaf = (nk.w & META_LEAF) != 0u;
        lk = T.nlink[node];
        push = !isleaf;
        if (isleaf) {
          for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) {
            if (dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c) < r2) {
              ++mine;
              hm = fmax(hm, T.h[s]);
              if (T.lbol[s] > 0.0) ++mylum;
            }
          }
        }
      }
    }
    if (out) {
      const uint32_t lbase = lum + wave_excl(mylum, lane);
      const uint32_t dbase = lum_total + (cnt - lum) + wave_excl(mine - mylum, lane);
      if (isleaf && mine) {
        uint32_t a = 0, b = 0;
        for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) {
          if (dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c) < r2) {
            if (T.lbol[s] > 0.0) out[lbase + a++] = s;
            else out[dbase + b++] = s;
          }
        }
      }
    }
    cnt += wave_sum_u(mine);
    lum += wave_sum_u(mylum);
    const uint64_t pm = ballot64(push);
    const int npush = __popcll(pm);
    if (sp + 2 * npush > kStackCap) {
      *overflow = true;
      break;
    }
    if (push) {
      const int ppos = mbcnt(pm);
      stack[sp + 2 * ppos] = lk.x;          // child 1
      stack[sp + 2 * ppos + 1] = node + 1u; // child 0
    }
    sp += 2 * npush;
    __syncthreads();
  }
  if (hmax) *hmax = wave_max(hm);
  if (nlum) *nlum = lum;
  return cnt;
}

// p-p radius (Section 2.4): past every bucket member by its size, then grown
// until no element inside is wider than the beam there (w r).  One
// wavefront per bucket.
__global__ void __launch_bounds__(64) k_setup(DevTree T, const uint32_t* blist,
                                              const uint32_t* nbp, double* brad, uint32_t* ncnt,
                                              uint32_t* nlumc) {
  const uint32_t b = blockIdx.x;
  if (b >= *nbp) return;
  __shared__ uint32_t stack[kStackCap];
  const int lane = threadIdx.x;
  const uint32_t leaf = blist[b];
  double c[3];
  leaf_centre(T, leaf, c);
  double r = 0.0;
  uint32_t cnt = 0, nlum = 0;
  bool overflow = false;
  if (T.flags & TREVR_NEAR_FIELD) {
    r = T.rpp_min;
    const uint2 lk = T.nlink[leaf];
    double rm = 0.0;
    for (uint32_t s = lk.x + lane; s < lk.x + lk.y; s += 64)
      rm = fmax(rm, sqrt(dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c)) + T.h[s]);
    r = fmax(r, wave_max(rm));
    for (;;) {
      double hm = 0.0;
      cnt = wave_near(T, c, r * r, stack, &hm, &nlum, nullptr, 0, &overflow);
      const double rn = fmax(r, hm / T.wbeam);
      if (!(rn > r) || overflow) break;
      r = rn;
    }
  }
  if (lane == 0) {
    brad[b] = r;
    ncnt[b] = cnt;
    nlumc[b] = nlum;
    if (overflow) atomicOr(T.err, ERR_STACK);
  }
}

__global__ void __launch_bounds__(64) k_near_fill(DevTree T, const uint32_t* blist,
                                                  const uint32_t* nbp, const double* brad,
                                                  const uint32_t* noff, const uint32_t* nlumc,
                                                  uint32_t* nidx) {
  const uint32_t b = blockIdx.x;
  if (b >= *nbp || !(T.flags & TREVR_NEAR_FIELD)) return;
  __shared__ uint32_t stack[kStackCap];
  double c[3];
  leaf_centre(T, blist[b], c);
  const double r = brad[b];
  bool overflow = false;
  wave_near(T, c, r * r, stack, nullptr, nullptr, nidx + noff[b], nlumc[b], &overflow);
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

// ------------------------------------------------------------- the walk
__global__ void __launch_bounds__(64) k_walk(DevTree T, const uint32_t* blist,
                                             const double* brad, uint32_t b0, uint32_t nbuck,
                                             uint2* cut, uint32_t* bstat) {
  const uint32_t bucket = b0 + blockIdx.x;
  if (bucket >= nbuck) return;
  __shared__ uint32_t stack[kStackCap];
  const int lane = threadIdx.x;
  const uint32_t leafb = blist[bucket];
  const double r = brad[bucket];
  const double r2 = r * r;
  double c[3];
  leaf_centre(T, leafb, c);
  uint2* out = cut + (size_t)blockIdx.x * kCutCap;
  uint32_t ncut = 0, nsrc = 0, ncells = 0;
  bool overflow = false;
  int sp = 1;
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
    if (valid) {
      nk = T.nk[node];
      cn = T.cen[node];
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
    if (sp + 2 * npush > kStackCap) {
      overflow = true;
      break;
    }
    if (push) {
      stack[sp + 2 * ppos] = T.nlink[node].x;      // child 1
      stack[sp + 2 * ppos + 1] = node + 1u;        // child 0
    }
    sp += 2 * npush;
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
      if (idx < kCutCap) out[idx] = make_uint2(node, meta);
    }
    ncut += (uint32_t)__popcll(wm);
    nsrc += (uint32_t)__popcll(ballot64(write && ((meta & 0xFFFFu) != CUT_NOPIX)));
    // element sources of opened luminous buckets, outside the p-p sphere
    uint64_t lm = ballot64(emit && opened && (nk.w & META_LUM));
    while (lm) {
      const int src_lane = __ffsll((long long)lm) - 1;
      lm &= lm - 1;
      const uint32_t lnode = (uint32_t)__shfl((int)node, src_lane);
      const uint2 lk = T.nlink[lnode];
      for (uint32_t base = 0; base < lk.y; base += 64) {
        const uint32_t s = lk.x + base + lane;
        bool is_src = false;
        uint32_t pix = 0u;
        if (base + lane < lk.y && T.lbol[s] > 0.0) {
          const double px = (double)T.x[s], py = (double)T.y[s], pz = (double)T.z[s];
          if (!(dist2_pt3(px, py, pz, c) < r2)) {
            is_src = true;
            pix = source_pixel(T.nside, px - c[0], py - c[1], pz - c[2]);
          }
        }
        const uint64_t sm = ballot64(is_src);
        if (is_src) {
          const uint32_t idx = ncut + (uint32_t)mbcnt(sm);
          if (idx < kCutCap) out[idx] = make_uint2(s, CUT_PART | pix);
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
    if (overflow) atomicOr(T.err, ERR_STACK);
    if (ncut > kCutCap) atomicOr(T.err, ERR_CUT);
    atomic_max_u64(&T.counters[CNT_MAX_CUT], ncut);
  }
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
// kNChunk elements at a time.  Elements are culled kSub at a time with FP32
// boxes (each element's position grown by its own size h, plus a margin),
// which is conservative: an element can only absorb on a line that passes
// within h of it.  Threads are mapped receiver-fastest, so the lines of a
// wavefront are nearly parallel and skip the same boxes.
constexpr int kSub = 16;
constexpr int kNSub = kNChunk / kSub;

template <int NB> struct NearTile {
  double x[kNChunk], y[kNChunk], z[kNChunk], h2[kNChunk];
  float sig[kNChunk], invh[kNChunk];
  float kap[kNChunk][NB];
  uint32_t slot[kNChunk];
  float blo[kNSub][3], bhi[kNSub][3];
};

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
    S.sig[t] = (float)(3.0 * (double)T.m[l] / (kPi * hl * hl));
    S.invh[t] = (float)(1.0 / hl);
#pragma unroll
    for (int b = 0; b < NB; ++b) S.kap[t][b] = T.kappa[(int64_t)b * T.n + l];
    S.slot[t] = l;
  }
  __syncthreads();
  if (t < kNSub) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int u1 = min((int)cl, (t + 1) * kSub);
    for (int u = t * kSub; u < u1; ++u) {
      const float h = sqrtf((float)S.h2[u]);
      const float p[3] = {(float)(S.x[u] - c[0]), (float)(S.y[u] - c[1]), (float)(S.z[u] - c[2])};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float m = h + 1e-5f * (fabsf(p[a]) + h);
        lo[a] = fminf(lo[a], p[a] - m);
        hi[a] = fmaxf(hi[a], p[a] + m);
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) { S.blo[t][a] = lo[a]; S.bhi[t][a] = hi[a]; }
  }
  __syncthreads();
}

// Next chunk of active bucket members (thread 0 keeps the cursor).
__device__ inline int load_receivers(const DevTree& T, const uint8_t* active, const double c[3],
                                     uint32_t& member, uint32_t mend, RecvInfo* recv,
                                     uint32_t* nrecv_s) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t k = 0;
    while (member < mend && k < (uint32_t)kRMax) {
      const uint32_t s = member++;
      if (active == nullptr || active[T.perm[s]]) {
        RecvInfo ri;
        ri.x[0] = (double)T.x[s];
        ri.x[1] = (double)T.y[s];
        ri.x[2] = (double)T.z[s];
        ri.h = T.h[s];
        for (int a = 0; a < 3; ++a) ri.rel[a] = (float)(ri.x[a] - c[a]);
        ri.inv_rh = (float)(1.0 / (kR * ri.h));
        ri.kfac = (float)(1.0 / (2.0 * ri.h * ri.h));
        ri.slot = s;
        recv[k++] = ri;
      }
    }
    *nrecv_s = k;
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

// For each receiver i and ray k: the optical depth of the p-p elements ahead
// of i on the ray (exact FP64 projection: a discontinuous decision) whose
// size h reaches the ray line (b < h, with b^2 = |d|^2 - proj^2: continuous,
// Sigma -> 0 at b = h): kappa_l Sigma_l(b), Sigma_l(b) = 3 m_l/(pi h_l^2)
// (1 - b/h_l).  Written to tpp[receiver][ray][band] for the far field.
template <int NB>
__global__ void __launch_bounds__(kNT) k_pp_rays(DevTree T, const uint32_t* blist,
                                                const uint32_t* noff, const uint32_t* nidx,
                                                const uint32_t* roff, uint32_t b0, uint32_t nbuck,
                                                const uint8_t* active, float* tpp) {
  const uint32_t bucket = b0 + blockIdx.x;
  if (bucket >= nbuck) return;
  const int t = threadIdx.x;
  __shared__ NearTile<NB> S;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s;
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0;
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  uint32_t rbase = roff[bucket];
  uint32_t member = lk.x;
  for (;;) {
    const int nrecv = load_receivers(T, active, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    const int stride = (kNT / nrecv) * nrecv;       // thread t keeps receiver t % nrecv
    const int gpr = (nray + 1) / 2;                 // two rays per thread
    const uint32_t P = (uint32_t)nrecv * (uint32_t)gpr;
    const int i = t % nrecv;
    const RecvInfo& ri = recv[i];
    for (uint32_t pb = 0; pb < P; pb += (uint32_t)stride) {
      const uint32_t p = pb + (uint32_t)t;
      const bool ok = t < stride && p < P;
      const int kb = ok ? 2 * (int)(p / nrecv) : 0;
      double nv[2][3];
      float of[3], inv[2][3];
      bool kok[2];
      float tau[2][NB];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        kok[q] = ok && kb + q < nray;
        const int kq = kok[q] ? kb + q : 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          nv[q][a] = T.ray_n[3 * kq + a];
          const float nf = (float)nv[q][a];
          inv[q][a] = (nf != 0.0f) ? 1.0f / nf : 1e30f;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) tau[q][b] = 0.0f;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) of[a] = ri.rel[a];
      const double xi0 = ri.x[0], xi1 = ri.x[1], xi2 = ri.x[2];
      const uint32_t si = ri.slot;
      for (uint32_t c0 = 0; c0 < nnear; c0 += kNChunk) {
        const uint32_t cl = min((uint32_t)kNChunk, nnear - c0);
        stage_near<NB>(S, T, near, c0, cl, c);
        const int nsub = ((int)cl + kSub - 1) / kSub;
        for (int sb = 0; sb < nsub; ++sb) {
          bool need = false;
          if (ok) {
            const float blo[3] = {S.blo[sb][0], S.blo[sb][1], S.blo[sb][2]};
            const float bhi[3] = {S.bhi[sb][0], S.bhi[sb][1], S.bhi[sb][2]};
            need = (kok[0] && ray_meets_box(of, inv[0], blo, bhi)) ||
                   (kok[1] && ray_meets_box(of, inv[1], blo, bhi));
          }
          if (ballot64(need) == 0ull) continue;
          if (!need) continue;
          const int u1 = min((int)cl, (sb + 1) * kSub);
          for (int u = sb * kSub; u < u1; ++u) {
            const double d0 = S.x[u] - xi0, d1 = S.y[u] - xi1, d2 = S.z[u] - xi2;
            const double dd = d0 * d0 + d1 * d1 + d2 * d2;
            const double h2 = S.h2[u];
            const bool other = S.slot[u] != si;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const double proj = d0 * nv[q][0] + d1 * nv[q][1] + d2 * nv[q][2];
              const double b2 = dd - proj * proj;
              if (proj > 0.0 && b2 < h2 && other && kok[q]) {
                const float bb = sqrtf((float)fmax(b2, 0.0));
                const float sg = S.sig[u] * (1.0f - bb * S.invh[u]);
#pragma unroll
                for (int b = 0; b < NB; ++b) tau[q][b] += S.kap[u][b] * sg;
              }
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (!kok[q]) continue;
        float* o = tpp + ((int64_t)(rbase + i) * nray + kb + q) * NB;
#pragma unroll
        for (int b = 0; b < NB; ++b) o[b] = tau[q][b];
      }
    }
    rbase += (uint32_t)nrecv;
  }
}

// For each receiver i and luminous p-p element j (i itself included, at
// r = 0): L_j K(r_ij, h_i) exp(-tau_ij), tau over the p-p elements closer to
// j than i is (exact FP64 squared distances: discontinuous) and within their
// size of the segment i-j (continuous).  J of i starts with the sum.
template <int NB>
__global__ void __launch_bounds__(kNT) k_pp_src(DevTree T, const uint32_t* blist,
                                               const uint32_t* noff, const uint32_t* nlumc,
                                               const uint32_t* nidx, uint32_t b0, uint32_t nbuck,
                                               const uint8_t* active, double* J) {
  const uint32_t bucket = b0 + blockIdx.x;
  if (bucket >= nbuck) return;
  const int t = threadIdx.x;
  __shared__ NearTile<NB> S;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s;
  __shared__ double red[kNT][NB];
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0, nl = nlumc[bucket];
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int64_t n = T.n;
  uint32_t member = lk.x;
  uint32_t nact = 0;
  for (;;) {
    const int nrecv = load_receivers(T, active, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    nact += (uint32_t)nrecv;
    const int stride = (kNT / nrecv) * nrecv;       // thread t keeps receiver t % nrecv
    const int i = t % nrecv;
    const RecvInfo& ri = recv[i];
    const double xi0 = ri.x[0], xi1 = ri.x[1], xi2 = ri.x[2];
    const uint32_t si = ri.slot;
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
      float tau[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) tau[b] = 0.0f;
      for (uint32_t c0 = 0; c0 < nnear; c0 += kNChunk) {
        const uint32_t cl = min((uint32_t)kNChunk, nnear - c0);
        stage_near<NB>(S, T, near, c0, cl, c);
        const int nsub = ((int)cl + kSub - 1) / kSub;
        for (int sb = 0; sb < nsub; ++sb) {
          bool need = false;
          if (ok && rij2 > 0.0) {
            float dmin2 = 0.0f;
            bool over = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const float lo = S.blo[sb][a], hi = S.bhi[sb][a];
              over = over && (smax[a] >= lo) && (smin[a] <= hi);
              const float dj = fmaxf(fmaxf(lo - jr[a], jr[a] - hi), 0.0f);
              dmin2 += dj * dj;
            }
            need = over && dmin2 < r2f;
          }
          if (ballot64(need) == 0ull) continue;
          if (!need) continue;
          const int u1 = min((int)cl, (sb + 1) * kSub);
          for (int u = sb * kSub; u < u1; ++u) {
            const double ux = S.x[u], uy = S.y[u], uz = S.z[u];
            const double f0 = ux - xj0, f1 = uy - xj1, f2 = uz - xj2;
            const double w0 = ux - xi0, w1 = uy - xi1, w2 = uz - xi2;
            double uu = (w0 * e0 + w1 * e1 + w2 * e2) * inv2;
            uu = fmin(1.0, fmax(0.0, uu));
            const double g0 = w0 - uu * e0, g1 = w1 - uu * e1, g2 = w2 - uu * e2;
            const double b2 = g0 * g0 + g1 * g1 + g2 * g2;
            const uint32_t us = S.slot[u];
            if ((f0 * f0 + f1 * f1 + f2 * f2 < rij2) && b2 < S.h2[u] && us != si && us != j) {
              const float bb = sqrtf((float)b2);
              const float sg = S.sig[u] * (1.0f - bb * S.invh[u]);
#pragma unroll
              for (int b = 0; b < NB; ++b) tau[b] += S.kap[u][b] * sg;
            }
          }
        }
      }
      if (ok) {
        const float Kv = fshape((float)sqrt(rij2) * ri.inv_rh) * ri.kfac;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[b] += (double)T.lum[(int64_t)b * n + j] * (double)Kv * exp(-(double)tau[b]);
      }
    }
    // receiver-wise sums in thread order (deterministic)
#pragma unroll
    for (int b = 0; b < NB; ++b) red[t][b] = acc[b];
    __syncthreads();
    if (t < nrecv * NB) {
      const int ii = t / NB, b = t % NB;
      double v = 0.0;
      for (int u = ii; u < stride; u += nrecv) v += red[u][b];
      J[(int64_t)b * n + T.perm[recv[ii].slot]] = v;
    }
  }
  if (t == 0) {
    atomicAdd(&T.counters[CNT_NEAR_PAIRS], (unsigned long long)nact * nnear);
    atomicAdd(&T.counters[CNT_NS_TRIPLES], (unsigned long long)nact * nl * nnear);
    atomic_max_u64(&T.counters[CNT_MAX_NEAR], (unsigned long long)nnear);
  }
}

// ------------------------------------------------------------- far field
// One workgroup of kFT threads per bucket.  Rays are taken in groups of 64;
// thread k < 64 owns ray k of the group (its sources and their optical
// depths), so hits update them without atomics.  Sources of a group are held
// kSrcCap at a time (a second window re-reads the cut; only very source-rich
// buckets need it).  Receivers are fixed per thread (t mod P2, P2 the power
// of two >= the receiver count), so each thread keeps one FP64 accumulator
// per band, reduced per receiver in a fixed order at the end.
constexpr int kFT = 256;
template <int NB> struct SrcCap { static constexpr int value = NB <= 4 ? 512 : 256; };

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

template <int NB>
__global__ void __launch_bounds__(kFT) k_far(DevTree T, const uint32_t* blist, const double* brad,
                                             const uint32_t* roff, uint32_t b0, uint32_t nbuck,
                                             const uint2* cut, const uint32_t* bstat,
                                             const float* tppg, const float* bg, double* J,
                                             const uint8_t* active) {
  constexpr int kSrcCap = SrcCap<NB>::value;
  const uint32_t bucket = b0 + blockIdx.x;
  if (bucket >= nbuck) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

  __shared__ float s_rel[kSrcCap][3];
  __shared__ float s_s[kSrcCap];
  __shared__ float s_tau[kSrcCap][NB];
  __shared__ float s_sfx[kSrcCap][NB];
  __shared__ float s_L[kSrcCap][NB];
  __shared__ uint8_t s_ray[kSrcCap];
  __shared__ uint16_t s_order[kSrcCap];
  __shared__ uint32_t ray_beg[65], ray_fill[64];
  __shared__ float tpp[kRMax][64][NB];
  __shared__ float tex[64][NB];
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, wcnt[kFT / 64], abs_count, cand_total;
  __shared__ double a_lo[64][3], a_hi[64][3];
  __shared__ float a_mc[64][3], a_d2[64], a_r2[64];
  __shared__ uint32_t a_node[64], a_pre[64];
  __shared__ unsigned long long a_mask[64];
  __shared__ double g_n[64][3], g_inv[64][3];
  __shared__ float g_nf[64][3];
  __shared__ double h_t0[kFT], h_t1[kFT];
  __shared__ uint32_t h_node[kFT], h_cnt[64], h_beg[65];
  __shared__ uint8_t h_ray[kFT];
  __shared__ uint16_t h_ord[kFT];
  __shared__ double red[kFT / 64][kRMax][NB];

  const uint32_t leafb = blist[bucket];
  const double r = brad[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t ncut = min(bstat[4 * bucket + 0], kCutCap);
  const uint2* mycut = cut + (size_t)blockIdx.x * kCutCap;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  const int ngroups = (nray + 63) / 64;
  const int64_t n = T.n;
  const bool use_bg = (T.flags & TREVR_BACKGROUND) && bg != nullptr;

  if (t == 0) abs_count = 0u;
  uint32_t nact_total = 0;
  uint32_t rbase = roff[bucket];
  uint32_t member = lk.x;
  for (;;) {
    const int nrecv = load_receivers(T, active, c, member, lk.x + lk.y, recv, &nrecv_s);
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
      int cls = 0;
      if (rt) {
        const int k = k0 + t;
        cls = T.ray_class[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double na = T.ray_n[3 * k + a];
          g_n[t][a] = na;
          g_inv[t][a] = (na != 0.0) ? 1.0 / na : 0.0;
          g_nf[t][a] = (float)na;
        }
      }
      for (int q = t; q < nrecv * kn; q += kFT) {
        const int i = q / kn, kq = q % kn;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          tpp[i][kq][b] = tppg[((int64_t)(rbase + i) * nray + k0 + kq) * NB + b];
      }

      for (uint32_t skip = 0;; skip += (uint32_t)kSrcCap) {
        // ---- sources whose pixel is in this group, window [skip, skip + cap)
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
          if (mine && gi >= skip && gi < skip + (uint32_t)kSrcCap) {
            const uint32_t slot = gi - skip;
            double p[3];
            float Lv[NB];
            if ((ent.y & CUT_KIND_MASK) == CUT_PART) {
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
              const double* nn = &T.ray_n[3 * pix];
              sd = v0 * nn[0] + v1 * nn[1] + v2 * nn[2];
            }
            s_rel[slot][0] = (float)v0;
            s_rel[slot][1] = (float)v1;
            s_rel[slot][2] = (float)v2;
            s_s[slot] = (float)sd;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              s_L[slot][b] = Lv[b];
              s_tau[slot][b] = 0.0f;
              s_sfx[slot][b] = 0.0f;
            }
            s_ray[slot] = (uint8_t)(pix - k0);
          }
          nsg_all += tot;
        }
        const uint32_t nsg = min(nsg_all - skip, (uint32_t)kSrcCap);
        // ---- bin sources by ray, then sort each ray's sources by distance
        if (t < 64) ray_fill[t] = 0u;
        __syncthreads();
        for (uint32_t q = t; q < nsg; q += kFT) atomicAdd(&ray_fill[s_ray[q]], 1u);
        __syncthreads();
        if (t < 64) {
          const uint32_t v = ray_fill[t];
          const uint32_t ex = wave_excl(v, t);
          ray_beg[t] = ex;
          if (t == 63) ray_beg[64] = ex + v;
          ray_fill[t] = ex;
        }
        __syncthreads();
        for (uint32_t q = t; q < nsg; q += kFT) {
          const uint32_t pos = atomicAdd(&ray_fill[s_ray[q]], 1u);
          s_order[pos] = (uint16_t)q;
        }
        __syncthreads();
        const uint32_t q0 = rt ? ray_beg[t] : 0u, q1 = rt ? ray_beg[t + 1] : 0u;
        for (uint32_t a = q0 + 1; a < q1; ++a) {     // insertion sort by s
          const uint16_t key = s_order[a];
          const float ks = s_s[key];
          uint32_t b = a;
          while (b > q0 && s_s[s_order[b - 1]] > ks) {
            s_order[b] = s_order[b - 1];
            --b;
          }
          s_order[b] = key;
        }

        // ---- cell absorption along each ray (Sections 2.5.1, 2.6).
        // Absorbing cut entries are staged 64 at a time; a conservative FP32
        // bounding-sphere test (rays split over the four wavefronts) gives each
        // its candidate rays; the (entry, ray) candidates are packed across
        // the block for the exact FP64 ray-box test; each hit is applied by the
        // thread owning its ray: sources on the ray inside the chord get the
        // partial length, the nearest source beyond it a suffix add (resolved
        // by a prefix sum over the ray's sources sorted by distance).
        float texl[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) texl[b] = 0.0f;
        uint32_t nabs = 0;
        for (uint32_t e0 = 0; e0 < ncut; e0 += 64) {
          if (t < 64) {
            const uint32_t e = e0 + (uint32_t)t;
            bool is = false;
            uint32_t node = 0;
            if (e < ncut) {
              const uint2 ent = mycut[e];
              is = (ent.y & CUT_ABS) != 0u;
              node = ent.x;
            }
            const uint64_t am = ballot64(is);
            if (t == 0) wcnt[0] = (uint32_t)__popcll(am);
            if (is) {
              const int pos = mbcnt(am);
              double lo[3], hi[3];
              node_box(T.hdr, T.nk[node], lo, hi);
              float R2 = 0.0f, D2 = 0.0f;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                a_lo[pos][a] = lo[a];
                a_hi[pos][a] = hi[a];
                const float m = (float)(0.5 * (lo[a] + hi[a]) - c[a]);
                const float hx = (float)(0.5 * (hi[a] - lo[a]));
                a_mc[pos][a] = m;
                R2 += hx * hx;
                D2 += m * m;
              }
              a_node[pos] = node;
              a_d2[pos] = D2;
              a_r2[pos] = R2;
              a_mask[pos] = 0ull;
            }
          }
          __syncthreads();
          const int na = (int)wcnt[0];
          {   // candidate rays: entry t%64, rays wv*16 .. wv*16+15
            const int ej = t & 63;
            if (ej < na) {
              const float D2 = a_d2[ej], R2 = a_r2[ej];
              const float marg = 1e-5f * D2 + 1e-30f;
              unsigned long long part = 0ull;
              const int ka = wv * 16, kb = min(kn, ka + 16);
              if (D2 - R2 <= marg) {
                for (int kq = ka; kq < kb; ++kq) part |= 1ull << kq;
              } else {
                const float thr = D2 - R2 - marg;
                const float m0 = a_mc[ej][0], m1 = a_mc[ej][1], m2 = a_mc[ej][2];
                for (int kq = ka; kq < kb; ++kq) {
                  const float nm = g_nf[kq][0] * m0 + g_nf[kq][1] * m1 + g_nf[kq][2] * m2;
                  if (nm > 0.0f && nm * nm >= thr) part |= 1ull << kq;
                }
              }
              if (part) atomicOr(&a_mask[ej], part);
            }
          }
          __syncthreads();
          if (t < 64) {
            const uint32_t cntc = (t < na) ? (uint32_t)__popcll(a_mask[t]) : 0u;
            const uint32_t pre = wave_excl(cntc, t);
            if (t < na) a_pre[t] = pre;
            if (t == 63) cand_total = pre + cntc;
          }
          __syncthreads();
          const uint32_t C = cand_total;
          for (uint32_t g0 = 0; g0 < C; g0 += kFT) {
            const uint32_t gi = g0 + (uint32_t)t;
            bool hit = false;
            double t0 = 0.0, t1 = 0.0;
            uint32_t hnode = 0;
            int kray = 0;
            if (gi < C) {
              int lo_j = 0, hi_j = na - 1;
              while (lo_j < hi_j) {
                const int mid = (lo_j + hi_j + 1) >> 1;
                if (a_pre[mid] <= gi) lo_j = mid; else hi_j = mid - 1;
              }
              uint64_t m = a_mask[lo_j];
              for (uint32_t rr = gi - a_pre[lo_j]; rr > 0; --rr) m &= m - 1ull;
              kray = __ffsll((long long)m) - 1;
              const double lo[3] = {a_lo[lo_j][0], a_lo[lo_j][1], a_lo[lo_j][2]};
              const double hi[3] = {a_hi[lo_j][0], a_hi[lo_j][1], a_hi[lo_j][2]};
              const double nn[3] = {g_n[kray][0], g_n[kray][1], g_n[kray][2]};
              const double iv[3] = {g_inv[kray][0], g_inv[kray][1], g_inv[kray][2]};
              double tin, tout;
              if (slab(lo, hi, c, nn, iv, tin, tout) && tout > fmax(tin, r)) {
                hit = true;
                t0 = fmax(tin, r);
                t1 = tout;
                hnode = a_node[lo_j];
              }
            }
            if (t < 64) h_cnt[t] = 0u;
            uint32_t nh;
            const uint32_t hp = block_compact(hit, wcnt, &nh);
            if (hit) {
              h_t0[hp] = t0;
              h_t1[hp] = t1;
              h_node[hp] = hnode;
              h_ray[hp] = (uint8_t)kray;
              atomicAdd(&h_cnt[kray], 1u);
            }
            __syncthreads();
            if (t < 64) {
              const uint32_t v = h_cnt[t];
              const uint32_t ex = wave_excl(v, t);
              h_beg[t] = ex;
              if (t == 63) h_beg[64] = ex + v;
              h_cnt[t] = ex;
            }
            __syncthreads();
            if (hit) h_ord[atomicAdd(&h_cnt[kray], 1u)] = (uint16_t)hp;
            __syncthreads();
            if (rt) {
              for (uint32_t hq = h_beg[t]; hq < h_beg[t + 1]; ++hq) {
                const int hi2 = h_ord[hq];
                const double ht0 = h_t0[hi2], ht1 = h_t1[hi2];
                const float len = (float)(ht1 - ht0);
                const float* al = &T.alpha[((int64_t)h_node[hi2] * T.nclass + cls) * NB];
                float av[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                  av[b] = al[b];
                  texl[b] += av[b] * len;
                }
                ++nabs;
                uint32_t lo_p = q0, hi_p = q1;     // first source beyond t0
                while (lo_p < hi_p) {
                  const uint32_t mid = (lo_p + hi_p) >> 1;
                  if ((double)s_s[s_order[mid]] > ht0) hi_p = mid; else lo_p = mid + 1;
                }
                uint32_t pq = lo_p;
                for (; pq < q1; ++pq) {
                  const uint32_t si = s_order[pq];
                  const double sq = (double)s_s[si];
                  if (!(sq < ht1)) break;
                  const float part = (float)(sq - ht0);
#pragma unroll
                  for (int b = 0; b < NB; ++b) s_tau[si][b] += av[b] * part;
                }
                if (pq < q1) {
                  const uint32_t si = s_order[pq];
#pragma unroll
                  for (int b = 0; b < NB; ++b) s_sfx[si][b] += av[b] * len;
                }
              }
            }
            __syncthreads();
          }
        }
        if (rt) {   // resolve the suffix adds along each ray
          float run[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) run[b] = 0.0f;
          for (uint32_t pq = q0; pq < q1; ++pq) {
            const uint32_t si = s_order[pq];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              run[b] += s_sfx[si][b];
              s_tau[si][b] += run[b];
            }
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) tex[t][b] = texl[b];
          if (skip == 0 && first_chunk) atomicAdd(&abs_count, nabs);
        }
        __syncthreads();

        // ---- far sources at every receiver (Section 2.5.1, eq. intint)
        if (has_i) {
          const RecvInfo& ri = recv[my_i];
          for (uint32_t q = (uint32_t)my_q; q < nsg; q += (uint32_t)per_round) {
            const float dx = s_rel[q][0] - ri.rel[0];
            const float dy = s_rel[q][1] - ri.rel[1];
            const float dz = s_rel[q][2] - ri.rel[2];
            const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
            const float Kv = fshape(rr * ri.inv_rh) * ri.kfac;
            const float ratio = rr * __builtin_amdgcn_rcpf(s_s[q]);
            const int ray = s_ray[q];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const float tau = s_tau[q][b];
              const float tc = (tau > 0.0f) ? tau * ratio : 0.0f;
              const float e = __expf(-(tpp[my_i][ray][b] + tc));
              acc[b] += (double)(s_L[q][b] * Kv * e);
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
    rbase += (uint32_t)nrecv;
  }

  __syncthreads();
  if (t == 0) {
    const uint32_t nsrc = bstat[4 * bucket + 1], ncells = bstat[4 * bucket + 2];
    const uint32_t nabs_total = abs_count;
    atomicAdd(&T.counters[CNT_BUCKETS], 1ull);
    atomicAdd(&T.counters[CNT_CELLS], (unsigned long long)ncells);
    atomicAdd(&T.counters[CNT_ABS], (unsigned long long)nabs_total);
    atomicAdd(&T.counters[CNT_SRC], (unsigned long long)nsrc);
    atomicAdd(&T.counters[CNT_SEG],
              (unsigned long long)nact_total * ((unsigned long long)nray + nabs_total + nsrc));
    atomicAdd(&T.counters[CNT_SRC_PAIRS], (unsigned long long)nact_total * nsrc);
  }
}

// ----------------------------------------------------- bucket ordering
// Buckets are processed heaviest first (a counting sort by the log2 of an
// estimate of their p-p work), so the slowest buckets start early instead of
// forming the tail of a launch.  Each bucket's result is independent of its
// position.
__global__ void k_cost_bins(const uint32_t* nbp, const uint32_t* bnact, const uint32_t* ncnt,
                            const uint32_t* nlumc, int nray, uint32_t* bbin, uint32_t* bins) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *nbp) return;
  const unsigned long long cost =
      (unsigned long long)bnact[b] * ((unsigned long long)ncnt[b] * (nray / 2 + nlumc[b]) + 2000ull);
  const int lg = 63 - __clzll((long long)cost);
  const uint32_t bin = (uint32_t)max(0, (kCostBins - 1) - min(lg, kCostBins - 1));
  bbin[b] = bin;
  atomicAdd(&bins[bin], 1u);
}

__global__ void k_bins_scan(uint32_t* bins) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int i = 0; i < kCostBins; ++i) {
    const uint32_t v = bins[i];
    bins[i] = run;
    run += v;
  }
}

__global__ void k_reorder(const uint32_t* nbp, const uint32_t* bbin, uint32_t* bins,
                          const uint32_t* blist, const uint32_t* bnact, const uint32_t* ncnt,
                          const uint32_t* nlumc, const double* brad, uint32_t* blist2,
                          uint32_t* bnact2, uint32_t* ncnt2, uint32_t* nlumc2, double* brad2) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *nbp) return;
  const uint32_t pos = atomicAdd(&bins[bbin[b]], 1u);
  blist2[pos] = blist[b];
  bnact2[pos] = bnact[b];
  ncnt2[pos] = ncnt[b];
  nlumc2[pos] = nlumc[b];
  brad2[pos] = brad[b];
}

// ============================================================ host side
struct Scratch {
  uint32_t *blist, *bnact, *ncnt, *nlumc, *roff, *bstat, *nb;
  uint32_t *blist2, *bnact2, *ncnt2, *nlumc2, *bbin, *bins;
  double *brad, *brad2;
  uint2* cut;
  uint32_t* nidx;
  float* tpp;
  size_t fixed;
};

static Scratch carve_scratch(void* base, int64_t nleaves) {
  Carve cv(base);
  Scratch s{};
  const int64_t L = std::max<int64_t>(nleaves, 1);
  s.nb = cv.take<uint32_t>(4);           // buckets, p-p total, active total
  s.blist = cv.take<uint32_t>(L);
  s.bnact = cv.take<uint32_t>(L + 1);
  s.ncnt = cv.take<uint32_t>(L + 1);
  s.nlumc = cv.take<uint32_t>(L);
  s.bstat = cv.take<uint32_t>(4 * L);
  s.brad = cv.take<double>(L);
  s.blist2 = cv.take<uint32_t>(L);
  s.bnact2 = cv.take<uint32_t>(L + 1);
  s.ncnt2 = cv.take<uint32_t>(L + 1);
  s.nlumc2 = cv.take<uint32_t>(L);
  s.brad2 = cv.take<double>(L);
  s.bbin = cv.take<uint32_t>(L);
  s.bins = cv.take<uint32_t>(kCostBins);
  s.cut = cv.take<uint2>((size_t)std::min<int64_t>(L, kBatch) * kCutCap);
  s.fixed = cv.off + 256;
  return s;
}

size_t scratch_fixed_bytes(int64_t n) { return carve_scratch(nullptr, n).fixed; }

template <int NB>
static void launch_pair(const DevTree& D, const Scratch& S, uint32_t b0, uint32_t nb, uint32_t cnt,
                        const float* bg, double* J, const uint8_t* active, hipStream_t st,
                        trevr_tree* T, trevr_status* rc) {
  hipEvent_t e0 = prof_begin(T);
  k_pp_rays<NB><<<cnt, kNT, 0, st>>>(D, S.blist, S.ncnt, S.nidx, S.bnact, b0, nb, active, S.tpp);
  *rc = hip_check(hipGetLastError(), "k_pp_rays");
  if (*rc != TREVR_OK) return;
  k_pp_src<NB><<<cnt, kNT, 0, st>>>(D, S.blist, S.ncnt, S.nlumc, S.nidx, b0, nb, active, J);
  *rc = hip_check(hipGetLastError(), "k_pp_src");
  if (*rc != TREVR_OK) return;
  prof_end(T, TREVR_PROF_NEAR, e0);
  hipEvent_t e1 = prof_begin(T);
  k_far<NB><<<cnt, kFT, 0, st>>>(D, S.blist, S.brad, S.bnact, b0, nb, S.cut, S.bstat, S.tpp, bg,
                                J, active);
  *rc = hip_check(hipGetLastError(), "k_far");
  prof_end(T, TREVR_PROF_REDUCE, e1);
}

trevr_status compute_J_impl(trevr_tree* T, const uint8_t* active, const float* bg, double* J,
                            void* scratch, size_t scratch_bytes) {
  hipStream_t st = T->stream;
  const int64_t nleaves = T->num_leaves;
  Scratch S = carve_scratch(scratch, nleaves);
  if (scratch_bytes < S.fixed) {
    T->scratch_needed = S.fixed;
    return set_error(TREVR_E_CAPACITY, "scratch smaller than its fixed part");
  }
  const DevTree& D = T->dev;
  trevr_status rc;
#define TREVR_LAUNCH_CHECK(what)                                               \
  do {                                                                         \
    if ((rc = hip_check(hipGetLastError(), what)) != TREVR_OK) return rc;      \
  } while (0)
  if ((rc = hip_check(hipMemsetAsync(T->buf.counters, 0, sizeof(unsigned long long) * CNT_N, st),
                      "memset counters")) != TREVR_OK) return rc;
  if ((rc = hip_check(hipMemsetAsync(S.nb, 0, sizeof(uint32_t) * 4, st), "memset")) != TREVR_OK)
    return rc;
  if ((rc = hip_check(hipMemsetAsync(S.ncnt, 0, sizeof(uint32_t) * (nleaves + 1), st), "memset")) !=
      TREVR_OK)
    return rc;
  if ((rc = hip_check(hipMemsetAsync(S.bnact, 0, sizeof(uint32_t) * (nleaves + 1), st), "memset")) !=
      TREVR_OK)
    return rc;
  hipEvent_t ev_setup = prof_begin(T);
  k_active_buckets<<<(unsigned)((T->num_nodes + 255) / 256), 256, 0, st>>>(D, active, S.blist,
                                                                            S.bnact, S.nb);
  TREVR_LAUNCH_CHECK("k_active_buckets");
  k_setup<<<(unsigned)nleaves, 64, 0, st>>>(D, S.blist, S.nb, S.brad, S.ncnt, S.nlumc);
  TREVR_LAUNCH_CHECK("k_setup");
  // heaviest buckets first
  if ((rc = hip_check(hipMemsetAsync(S.bins, 0, sizeof(uint32_t) * kCostBins, st), "memset")) != TREVR_OK)
    return rc;
  if ((rc = hip_check(hipMemsetAsync(S.ncnt2, 0, sizeof(uint32_t) * (nleaves + 1), st), "memset")) != TREVR_OK)
    return rc;
  if ((rc = hip_check(hipMemsetAsync(S.bnact2, 0, sizeof(uint32_t) * (nleaves + 1), st), "memset")) != TREVR_OK)
    return rc;
  k_cost_bins<<<(unsigned)((nleaves + 255) / 256), 256, 0, st>>>(S.nb, S.bnact, S.ncnt, S.nlumc,
                                                                 T->nray, S.bbin, S.bins);
  TREVR_LAUNCH_CHECK("k_cost_bins");
  k_bins_scan<<<1, 64, 0, st>>>(S.bins);
  TREVR_LAUNCH_CHECK("k_bins_scan");
  k_reorder<<<(unsigned)((nleaves + 255) / 256), 256, 0, st>>>(
      S.nb, S.bbin, S.bins, S.blist, S.bnact, S.ncnt, S.nlumc, S.brad, S.blist2, S.bnact2, S.ncnt2,
      S.nlumc2, S.brad2);
  TREVR_LAUNCH_CHECK("k_reorder");
  std::swap(S.blist, S.blist2);
  std::swap(S.bnact, S.bnact2);
  std::swap(S.ncnt, S.ncnt2);
  std::swap(S.nlumc, S.nlumc2);
  std::swap(S.brad, S.brad2);
  k_scan_u32<<<1, 1024, 0, st>>>(S.ncnt, nleaves + 1, S.nb + 1);
  TREVR_LAUNCH_CHECK("k_scan_u32");
  k_scan_u32<<<1, 1024, 0, st>>>(S.bnact, nleaves + 1, S.nb + 2);
  TREVR_LAUNCH_CHECK("k_scan_u32");
  uint32_t* hbuf = T->host_u32;
  hipError_t e = hipMemcpyAsync(hbuf, S.nb, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if ((rc = hip_check(e, "bucket readback")) != TREVR_OK) return rc;
  const uint32_t nb = hbuf[0], near_total = hbuf[1], act_total = hbuf[2];
  const size_t near_off = (S.fixed + 255) & ~(size_t)255;
  const size_t tpp_off = (near_off + sizeof(uint32_t) * (size_t)near_total + 255) & ~(size_t)255;
  const size_t need = tpp_off + sizeof(float) * (size_t)act_total * T->nray * T->B + 256;
  T->scratch_needed = need;
  if (scratch_bytes < need) return set_error(TREVR_E_CAPACITY, "scratch too small for the p-p lists");
  S.nidx = (uint32_t*)((char*)scratch + near_off);
  S.tpp = (float*)((char*)scratch + tpp_off);
  if (nb > 0) {
    k_near_fill<<<nb, 64, 0, st>>>(D, S.blist, S.nb, S.brad, S.ncnt, S.nlumc, S.nidx);
    TREVR_LAUNCH_CHECK("k_near_fill");
  }
  prof_end(T, TREVR_PROF_SETUP, ev_setup);
  for (uint32_t b0 = 0; b0 < nb; b0 += kBatch) {
    const uint32_t cnt = std::min<uint32_t>(kBatch, nb - b0);
    hipEvent_t ev_walk = prof_begin(T);
    k_walk<<<cnt, 64, 0, st>>>(D, S.blist, S.brad, b0, nb, S.cut, S.bstat);
    TREVR_LAUNCH_CHECK("k_walk");
    prof_end(T, TREVR_PROF_WALK, ev_walk);
    switch (T->B) {
      case 1: launch_pair<1>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 2: launch_pair<2>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 3: launch_pair<3>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 4: launch_pair<4>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 5: launch_pair<5>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 6: launch_pair<6>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      case 7: launch_pair<7>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
      default: launch_pair<8>(D, S, b0, nb, cnt, bg, J, active, st, T, &rc); break;
    }
    if (rc != TREVR_OK) return rc;
  }
#undef TREVR_LAUNCH_CHECK
  T->counters_valid = true;
  return TREVR_OK;
}

}  // namespace trevr
