// Mean intensity J at active elements on gfx950 (Sections 2.1-2.6 of
// Wadsley, Baumschlager & Shen 2023).
//
// Per active bucket (a leaf of the radiation tree holding >= 1 active
// element) the work is split over kernels:
//   k_active_buckets  list buckets with active members;
//   k_setup           p-p radius by fixed point and the p-p set size;
//   k_near_fill       the p-p set (sorted slots) in key order;
//   k_walk            one wavefront walks the tree cooperatively (LDS stack,
//                     ballot compaction) and writes the bucket's cut: accepted
//                     cells, opened buckets and resolved element sources, each
//                     source tagged with its HEALPix pixel;
//   k_reduce          one wavefront reduces the cut ray by ray: rays are taken
//                     in groups of 64 with one lane per ray, so each lane owns
//                     its ray's sources and adds the optical depth of every
//                     absorbing cell its ray crosses without atomics; then the
//                     lanes sweep the sources against every receiver,
//                     accumulating J in FP64.
// Decisions (opening test, p-p membership, pixel of a source, ray-box
// intersection) are made in FP64 with the same correctly rounded operation
// sequence as their definition, so they are reproducible; transcendental
// physics (exp, the intensity kernel) runs in FP32 with FP64 accumulation.

#include <algorithm>
#include <cmath>

#include "trevr_internal.hpp"

namespace trevr {

constexpr int kRMax = 8;        // receivers per pass
constexpr int kStackCap = 3072; // walk stack entries
constexpr int kNearSrcCap = 512;
constexpr uint32_t kCutCap = 2048;
constexpr uint32_t kBatch = 16384;

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

// Elements strictly within sqrt(r2) of c: count, largest size, and
// optionally their slots in key order.  Boxes are pruned conservatively
// (an element may sit an ulp outside its box after quantisation).
__device__ inline uint32_t near_scan(const DevTree& T, const double c[3], double r2,
                                     double* hmax, uint32_t* out) {
  uint32_t cnt = 0;
  double hm = 0.0;
  const double prune = r2 * (1.0 + 1e-9);
  int64_t node = 0;
  while (node < T.num_nodes) {
    const uint4 nk = T.nk[node];
    double lo[3], hi[3];
    node_box(T.hdr, nk, lo, hi);
    if (dist2_box(lo, hi, c) > prune) {
      node = T.next[node];
      continue;
    }
    if (nk.w & META_LEAF) {
      const uint2 lk = T.nlink[node];
      for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) {
        if (dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c) < r2) {
          if (out) out[cnt] = s;
          ++cnt;
          hm = fmax(hm, T.h[s]);
        }
      }
    }
    ++node;
  }
  if (hmax) *hmax = hm;
  return cnt;
}

// p-p radius (Section 2.4): past every bucket member by its size, then grown
// until no element inside is wider than the beam there (w r).
__global__ void k_setup(DevTree T, const uint32_t* blist, const uint32_t* nbp, double* brad,
                        uint32_t* ncnt) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *nbp) return;
  const uint32_t leaf = blist[b];
  double c[3];
  leaf_centre(T, leaf, c);
  double r = 0.0;
  uint32_t cnt = 0;
  if (T.flags & TREVR_NEAR_FIELD) {
    r = T.rpp_min;
    const uint2 lk = T.nlink[leaf];
    for (uint32_t s = lk.x; s < lk.x + lk.y; ++s)
      r = fmax(r, sqrt(dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c)) + T.h[s]);
    for (;;) {
      double hm = 0.0;
      cnt = near_scan(T, c, r * r, &hm, nullptr);
      const double rn = fmax(r, hm / T.wbeam);
      if (!(rn > r)) break;
      r = rn;
    }
  }
  brad[b] = r;
  ncnt[b] = cnt;
}

__global__ void k_near_fill(DevTree T, const uint32_t* blist, const uint32_t* nbp,
                            const double* brad, const uint32_t* noff, uint32_t* nidx) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *nbp) return;
  if (!(T.flags & TREVR_NEAR_FIELD)) return;
  double c[3];
  leaf_centre(T, blist[b], c);
  const double r = brad[b];
  near_scan(T, c, r * r, nullptr, nidx + noff[b]);
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
  const float y2 = 1.0f / (x * x);
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

struct RecvInfo {
  double x[3];
  double h;
  float rel[3];    // position relative to the bucket centre
  float inv_rh;    // 1/(R h)
  float kfac;      // 1/(2 h^2)
  uint32_t slot;
};

// ---------------------------------------------------------- the reduction
// Sources of one ray group held on chip.
template <int NB> struct SrcCap { static constexpr int value = NB <= 3 ? 1024 : 512; };

template <int NB>
__global__ void __launch_bounds__(64) k_reduce(DevTree T, const uint32_t* blist,
                                               const double* brad, const uint32_t* noff,
                                               const uint32_t* nidx, uint32_t b0,
                                               uint32_t nbuck, const uint2* cut,
                                               const uint32_t* bstat, const float* bg,
                                               double* J, uint8_t const* active) {
  constexpr int kSrcCap = SrcCap<NB>::value;
  const uint32_t bucket = b0 + blockIdx.x;
  if (bucket >= nbuck) return;
  const int lane = threadIdx.x;

  __shared__ float s_rel[kSrcCap][3];
  __shared__ float s_s[kSrcCap];
  __shared__ float s_tau[kSrcCap][NB];
  __shared__ float s_L[kSrcCap][NB];
  __shared__ uint8_t s_ray[kSrcCap];
  __shared__ uint16_t s_order[kSrcCap];
  __shared__ uint32_t ray_beg[65];
  __shared__ uint32_t ray_fill[64];
  __shared__ float tpp[kRMax][64][NB];
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nsrc_list[kNearSrcCap];

  const uint32_t leafb = blist[bucket];
  const double r = brad[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t ncut = min(bstat[4 * bucket + 0], kCutCap);
  const uint2* mycut = cut + (size_t)blockIdx.x * kCutCap;
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0;
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  const int ngroups = (nray + 63) / 64;
  const int64_t n = T.n;
  const bool use_bg = (T.flags & TREVR_BACKGROUND) && bg != nullptr;
  constexpr double kR = 0.48860251190291992;   // (3/(4 pi))^(1/2)

  uint32_t nabs_total = 0;
  uint32_t nact_total = 0;
  uint32_t member = lk.x;
  const uint32_t mend = lk.x + lk.y;
  while (true) {
    // next chunk of active receivers
    __shared__ uint32_t nrecv_s;
    if (lane == 0) {
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
      nrecv_s = k;
    }
    member = (uint32_t)__shfl((int)member, 0);
    __syncthreads();
    const int nrecv = (int)nrecv_s;
    if (nrecv == 0) break;
    const bool first_chunk = nact_total == 0;
    nact_total += (uint32_t)nrecv;

    double acc[kRMax][NB];
#pragma unroll
    for (int i = 0; i < kRMax; ++i)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[i][b] = 0.0;

    for (int g = 0; g < ngroups; ++g) {
      const int k0 = 64 * g;
      const int kn = min(64, nray - k0);
      const int k = k0 + lane;
      const bool rlane = lane < kn;
      double nv[3] = {0.0, 0.0, 1.0}, inv[3] = {0.0, 0.0, 0.0};
      int cls = 0;
      if (rlane) {
        for (int a = 0; a < 3; ++a) {
          nv[a] = T.ray_n[3 * k + a];
          inv[a] = (nv[a] != 0.0) ? 1.0 / nv[a] : 0.0;
        }
        cls = T.ray_class[k];
      }
      // ---- p-p optical depth along each ray from each receiver (Section 2.4)
      if (rlane) {
        for (int i = 0; i < nrecv; ++i) {
          const RecvInfo ri = recv[i];
          double tau[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) tau[b] = 0.0;
          for (uint32_t q = 0; q < nnear; ++q) {
            const uint32_t l = near[q];
            if (l == ri.slot) continue;
            const double d0 = (double)T.x[l] - ri.x[0];
            const double d1 = (double)T.y[l] - ri.x[1];
            const double d2 = (double)T.z[l] - ri.x[2];
            const double proj = d0 * nv[0] + d1 * nv[1] + d2 * nv[2];
            if (!(proj > 0.0)) continue;
            const double cx = d1 * nv[2] - d2 * nv[1];
            const double cy = d2 * nv[0] - d0 * nv[2];
            const double cz = d0 * nv[1] - d1 * nv[0];
            const double bb = sqrt(cx * cx + cy * cy + cz * cz);
            const double hl = T.h[l];
            if (!(bb < hl)) continue;
            const double sig = (3.0 * (double)T.m[l] / (kPi * hl * hl)) * (1.0 - bb / hl);
#pragma unroll
            for (int b = 0; b < NB; ++b) tau[b] += (double)T.kappa[(int64_t)b * n + l] * sig;
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) tpp[i][lane][b] = (float)tau[b];
        }
      }

      // Sources of this group are held kSrcCap at a time; a second window
      // re-reads the cut, which only very source-rich buckets need.
      for (uint32_t skip = 0;; skip += (uint32_t)kSrcCap) {
        // ---- sources whose pixel is in this group, window [skip, skip + cap)
        uint32_t nsg_all = 0;
        for (uint32_t e0 = 0; e0 < ncut; e0 += 64) {
          const uint32_t e = e0 + lane;
          bool mine = false;
          uint2 ent = make_uint2(0, 0);
          uint32_t pix = CUT_NOPIX;
          if (e < ncut) {
            ent = mycut[e];
            pix = ent.y & 0xFFFFu;
            mine = pix != CUT_NOPIX && (int)pix >= k0 && (int)pix < k0 + kn;
          }
          const uint64_t m = ballot64(mine);
          if (mine) {
            const uint32_t gi = nsg_all + (uint32_t)mbcnt(m);
            if (gi >= skip && gi < skip + (uint32_t)kSrcCap) {
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
              double s = 0.0;
              if (!(v0 == 0.0 && v1 == 0.0 && v2 == 0.0)) {
                const double* nn = &T.ray_n[3 * pix];
                s = v0 * nn[0] + v1 * nn[1] + v2 * nn[2];
              }
              s_rel[slot][0] = (float)v0;
              s_rel[slot][1] = (float)v1;
              s_rel[slot][2] = (float)v2;
              s_s[slot] = (float)s;
  #pragma unroll
              for (int b = 0; b < NB; ++b) {
                s_L[slot][b] = Lv[b];
                s_tau[slot][b] = 0.0f;
              }
              s_ray[slot] = (uint8_t)(pix - k0);
            }
          }
          nsg_all += (uint32_t)__popcll(m);
        }
        const uint32_t nsg = min(nsg_all - skip, (uint32_t)kSrcCap);
        // ---- bin sources by ray
        ray_fill[lane] = 0u;
        __syncthreads();
        for (uint32_t q = lane; q < nsg; q += 64) atomicAdd(&ray_fill[s_ray[q]], 1u);
        __syncthreads();
        {
          uint32_t v = ray_fill[lane];
          uint32_t incl = v;
  #pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)incl, o);
            if (lane >= o) incl += u;
          }
          ray_beg[lane] = incl - v;
          if (lane == 63) ray_beg[64] = incl;
          ray_fill[lane] = incl - v;
        }
        __syncthreads();
        for (uint32_t q = lane; q < nsg; q += 64) {
          const uint32_t pos = atomicAdd(&ray_fill[s_ray[q]], 1u);
          s_order[pos] = (uint16_t)q;
        }
        __syncthreads();

        // ---- cell absorption along each ray (Sections 2.5.1, 2.6)
        float texl[NB];
  #pragma unroll
        for (int b = 0; b < NB; ++b) texl[b] = 0.0f;
        uint32_t nabs = 0;
        const uint32_t q0 = rlane ? ray_beg[lane] : 0u, q1 = rlane ? ray_beg[lane + 1] : 0u;
        for (uint32_t e = 0; e < ncut; ++e) {
          const uint2 ent = mycut[e];
          if (!(ent.y & CUT_ABS)) continue;
          double lo[3], hi[3];
          node_box(T.hdr, T.nk[ent.x], lo, hi);
          double tin, tout;
          if (rlane && slab(lo, hi, c, nv, inv, tin, tout) && tout > fmax(tin, r)) {
            const double t0 = fmax(tin, r);
            ++nabs;
            const float* al = &T.alpha[((int64_t)ent.x * T.nclass + cls) * NB];
            float a[NB];
  #pragma unroll
            for (int b = 0; b < NB; ++b) {
              a[b] = al[b];
              texl[b] += a[b] * (float)(tout - t0);
            }
            for (uint32_t q = q0; q < q1; ++q) {
              const uint32_t si = s_order[q];
              const double s = (double)s_s[si];
              if (!(s > t0)) continue;
              const float len = (float)(fmin(tout, s) - t0);
  #pragma unroll
              for (int b = 0; b < NB; ++b) s_tau[si][b] += a[b] * len;
            }
          }
        }
        if (skip == 0 && first_chunk) nabs_total += wave_sum_u(nabs);
        __syncthreads();

        // ---- far sources at every receiver (Section 2.5.1, eq. intint)
        for (uint32_t q = lane; q < nsg; q += 64) {
          const float sx = s_rel[q][0], sy = s_rel[q][1], sz = s_rel[q][2];
          const float ss = s_s[q];
          const int ray = s_ray[q];
          float tau[NB], Lv[NB];
  #pragma unroll
          for (int b = 0; b < NB; ++b) { tau[b] = s_tau[q][b]; Lv[b] = s_L[q][b]; }
  #pragma unroll
          for (int i = 0; i < kRMax; ++i) {
            if (i < nrecv) {
              const float dx = sx - recv[i].rel[0], dy = sy - recv[i].rel[1], dz = sz - recv[i].rel[2];
              const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
              const float Kv = fshape(rr * recv[i].inv_rh) * recv[i].kfac;
              const float ratio = rr / ss;
  #pragma unroll
              for (int b = 0; b < NB; ++b) {
                const float tc = (tau[b] > 0.0f) ? tau[b] * ratio : 0.0f;
                const float e = __expf(-(tpp[i][ray][b] + tc));
                acc[i][b] += (double)(Lv[b] * Kv * e);
              }
            }
          }
        }
        // ---- isotropic background along each ray (to the root-cube edge)
        if (use_bg && rlane && skip == 0) {
  #pragma unroll
          for (int i = 0; i < kRMax; ++i)
            if (i < nrecv)
  #pragma unroll
              for (int b = 0; b < NB; ++b)
                acc[i][b] += (4.0 * kPi / nray) * (double)bg[b] *
                             (double)__expf(-(tpp[i][lane][b] + texl[b]));
        }
        __syncthreads();
        if (nsg_all <= skip + (uint32_t)kSrcCap) break;
      }
      __syncthreads();
    }

    // ---- p-p sources, the receiver itself included (Section 2.4); the
    // luminous members of the p-p set are taken kNearSrcCap at a time
    for (uint32_t c0 = 0; c0 < nnear; c0 += (uint32_t)kNearSrcCap) {
      const uint32_t c1 = min(nnear, c0 + (uint32_t)kNearSrcCap);
      uint32_t nns = 0;
      for (uint32_t q0 = c0; q0 < c1; q0 += 64) {
        const uint32_t q = q0 + lane;
        const bool is = q < c1 && T.lbol[near[q]] > 0.0;
        const uint64_t m = ballot64(is);
        if (is) nsrc_list[nns + (uint32_t)mbcnt(m)] = near[q];
        nns += (uint32_t)__popcll(m);
      }
      __syncthreads();
      for (uint32_t pq = lane; pq < (uint32_t)nrecv * nns; pq += 64) {
        const int i = (int)(pq / nns);
        const uint32_t j = nsrc_list[pq % nns];
        const RecvInfo ri = recv[i];
        const double xj0 = (double)T.x[j], xj1 = (double)T.y[j], xj2 = (double)T.z[j];
        const double e0 = xj0 - ri.x[0], e1 = xj1 - ri.x[1], e2 = xj2 - ri.x[2];
        const double rij2 = e0 * e0 + e1 * e1 + e2 * e2;
        double tau[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) tau[b] = 0.0;
        for (uint32_t q = 0; q < nnear; ++q) {
          const uint32_t l = near[q];
          if (l == ri.slot || l == j) continue;
          const double xl0 = (double)T.x[l], xl1 = (double)T.y[l], xl2 = (double)T.z[l];
          const double f0 = xl0 - xj0, f1 = xl1 - xj1, f2 = xl2 - xj2;
          if (!(f0 * f0 + f1 * f1 + f2 * f2 < rij2)) continue;
          const double w0 = xl0 - ri.x[0], w1 = xl1 - ri.x[1], w2 = xl2 - ri.x[2];
          double u = (w0 * e0 + w1 * e1 + w2 * e2) / rij2;
          u = fmin(1.0, fmax(0.0, u));
          const double g0 = w0 - u * e0, g1 = w1 - u * e1, g2 = w2 - u * e2;
          const double bb = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
          const double hl = T.h[l];
          if (!(bb < hl)) continue;
          const double sig = (3.0 * (double)T.m[l] / (kPi * hl * hl)) * (1.0 - bb / hl);
#pragma unroll
          for (int b = 0; b < NB; ++b) tau[b] += (double)T.kappa[(int64_t)b * n + l] * sig;
        }
        const float rij = (float)sqrt(rij2);
        const float Kv = fshape(rij * ri.inv_rh) * ri.kfac;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double v = (double)T.lum[(int64_t)b * n + j] * (double)Kv * exp(-tau[b]);
#pragma unroll
          for (int ii = 0; ii < kRMax; ++ii)
            if (ii == i) acc[ii][b] += v;
        }
      }
      __syncthreads();
    }

    // ---- reduce over lanes, thick-element correction (Section 2.1), store
#pragma unroll
    for (int i = 0; i < kRMax; ++i) {
      if (i >= nrecv) continue;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double v = wave_sum(acc[i][b]);
        if (lane == b) {
          const uint32_t s = recv[i].slot;
          double out = v;
          if (T.flags & TREVR_THICK_CORR) {
            const double tau = (double)T.kappa[(int64_t)b * n + s] * (double)T.rho[s] * recv[i].h;
            out *= (tau == 0.0) ? 1.0 : -expm1(-tau) / tau;
          }
          J[(int64_t)b * n + T.perm[s]] = out;
        }
      }
    }
    __syncthreads();
  }

  if (lane == 0) {
    const uint32_t nsrc = bstat[4 * bucket + 1], ncells = bstat[4 * bucket + 2];
    atomicAdd(&T.counters[CNT_BUCKETS], 1ull);
    atomicAdd(&T.counters[CNT_CELLS], (unsigned long long)ncells);
    atomicAdd(&T.counters[CNT_ABS], (unsigned long long)nabs_total);
    atomicAdd(&T.counters[CNT_SRC], (unsigned long long)nsrc);
    atomicAdd(&T.counters[CNT_SEG],
              (unsigned long long)nact_total * ((unsigned long long)nray + nabs_total + nsrc));
    atomicAdd(&T.counters[CNT_NEAR_PAIRS], (unsigned long long)nact_total * nnear);
    atomic_max_u64(&T.counters[CNT_MAX_NEAR], (unsigned long long)nnear);
  }
}

// ============================================================ host side
struct Scratch {
  uint32_t *blist, *bnact, *ncnt, *bstat, *nb, *near_total;
  double* brad;
  uint2* cut;
  uint32_t* nidx;
  size_t fixed;
};

static Scratch carve_scratch(void* base, int64_t n, int64_t nleaves) {
  Carve cv(base);
  Scratch s{};
  const int64_t L = std::max<int64_t>(nleaves, 1);
  s.nb = cv.take<uint32_t>(4);
  s.near_total = s.nb + 1;
  s.blist = cv.take<uint32_t>(L);
  s.bnact = cv.take<uint32_t>(L);
  s.ncnt = cv.take<uint32_t>(L + 1);
  s.bstat = cv.take<uint32_t>(4 * L);
  s.brad = cv.take<double>(L);
  s.cut = cv.take<uint2>((size_t)std::min<int64_t>(L, kBatch) * kCutCap);
  s.fixed = cv.off + 256;
  s.nidx = cv.take<uint32_t>(0);
  (void)n;
  return s;
}

size_t scratch_fixed_bytes(int64_t n) { return carve_scratch(nullptr, n, n).fixed; }

template <int NB>
static void launch_reduce(const DevTree& D, const Scratch& S, uint32_t b0, uint32_t nb,
                          uint32_t cnt, const float* bg, double* J, const uint8_t* active,
                          hipStream_t st) {
  k_reduce<NB><<<cnt, 64, 0, st>>>(D, S.blist, S.brad, S.ncnt, S.nidx, b0, nb, S.cut, S.bstat,
                                   bg, J, active);
}

trevr_status compute_J_impl(trevr_tree* T, const uint8_t* active, const float* bg, double* J,
                            void* scratch, size_t scratch_bytes) {
  hipStream_t st = T->stream;
  const int64_t nleaves = T->num_leaves;
  Scratch S = carve_scratch(scratch, T->n, nleaves);
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
  k_active_buckets<<<(unsigned)((T->num_nodes + 255) / 256), 256, 0, st>>>(D, active, S.blist,
                                                                            S.bnact, S.nb);
  TREVR_LAUNCH_CHECK("k_active_buckets");
  k_setup<<<(unsigned)((nleaves + 63) / 64), 64, 0, st>>>(D, S.blist, S.nb, S.brad, S.ncnt);
  TREVR_LAUNCH_CHECK("k_setup");
  k_scan_u32<<<1, 1024, 0, st>>>(S.ncnt, nleaves + 1, S.near_total);
  TREVR_LAUNCH_CHECK("k_scan_inplace");
  uint32_t* hbuf = nullptr;
  if ((rc = hip_check(hipHostMalloc((void**)&hbuf, 2 * sizeof(uint32_t)), "hipHostMalloc")) != TREVR_OK)
    return rc;
  hipError_t e = hipMemcpyAsync(hbuf, S.nb, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const uint32_t nb = hbuf[0], near_total = hbuf[1];
  (void)hipHostFree(hbuf);
  if ((rc = hip_check(e, "bucket readback")) != TREVR_OK) return rc;
  const size_t need = S.fixed + sizeof(uint32_t) * (size_t)near_total + 256;
  T->scratch_needed = need;
  if (scratch_bytes < need) return set_error(TREVR_E_CAPACITY, "scratch too small for the p-p lists");
  S.nidx = (uint32_t*)((char*)scratch + ((S.fixed + 255) & ~(size_t)255));
  if (nb > 0) {
    k_near_fill<<<(unsigned)((nb + 63) / 64), 64, 0, st>>>(D, S.blist, S.nb, S.brad, S.ncnt, S.nidx);
    TREVR_LAUNCH_CHECK("k_near_fill");
  }
  for (uint32_t b0 = 0; b0 < nb; b0 += kBatch) {
    const uint32_t cnt = std::min<uint32_t>(kBatch, nb - b0);
    k_walk<<<cnt, 64, 0, st>>>(D, S.blist, S.brad, b0, nb, S.cut, S.bstat);
    TREVR_LAUNCH_CHECK("k_walk");
    switch (T->B) {
      case 1: launch_reduce<1>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 2: launch_reduce<2>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 3: launch_reduce<3>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 4: launch_reduce<4>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 5: launch_reduce<5>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 6: launch_reduce<6>(D, S, b0, nb, cnt, bg, J, active, st); break;
      case 7: launch_reduce<7>(D, S, b0, nb, cnt, bg, J, active, st); break;
      default: launch_reduce<8>(D, S, b0, nb, cnt, bg, J, active, st); break;
    }
    TREVR_LAUNCH_CHECK("k_reduce");
  }
#undef TREVR_LAUNCH_CHECK
  T->counters_valid = true;
  return TREVR_OK;
}

}  // namespace trevr
