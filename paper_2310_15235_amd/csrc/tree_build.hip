// Radiation tree construction on gfx950 (Section 2.3 and 2.6 of Wadsley,
// Baumschlager & Shen 2023): root cube, 63-bit Morton keys (21 bits per
// axis, x first), stable LSD radix sort, a radix tree whose nodes split at
// the first differing key bit (half-way along the longest axis of a cube or
// 2:1 box) down to buckets of at most leaf_size elements, node moments
// (luminosities, luminosity centre, bucket absorption) and per-direction
// transmission-averaged absorption.
//
// Levels are built top-down, one launch per level (children of a level are
// allocated with an atomic counter), then renumbered into depth-first
// preorder so a subtree is a contiguous index range.  Moments and
// transmission tables are reduced bottom-up, level by level, with FP64 sums
// formed in a fixed order (buckets sum their elements in key order; a parent
// adds its two children), which makes every node moment independent of the
// launch shape.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "trevr_internal.hpp"

namespace trevr {

// --------------------------------------------------------------- helpers
__device__ inline uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ inline bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

// ------------------------------------------------------------- root cube
__global__ void k_init(uint32_t* bbox_u, uint32_t* err, unsigned long long* counters,
                       uint32_t* alloc) {
  const int t = threadIdx.x;
  if (t < 3) { bbox_u[t] = 0xFFFFFFFFu; bbox_u[3 + t] = 0u; }
  if (t < 4) err[t] = 0u;
  if (t < CNT_N) counters[t] = 0ull;
  if (t == 0) *alloc = 1u;
}

__global__ void __launch_bounds__(256) k_bbox(const float* x, const float* y, const float* z,
                                              int64_t n, uint32_t* bbox_u) {
  uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v[3] = {f2ord(x[i]), f2ord(y[i]), f2ord(z[i])};
#pragma unroll
    for (int a = 0; a < 3; ++a) { mn[a] = min(mn[a], v[a]); mx[a] = max(mx[a], v[a]); }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], o));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], o));
    }
  }
  // per workgroup, then one set of atomics (the six words share a cache line,
  // so atomics on them queue behind one another)
  __shared__ uint32_t part[4][6];
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      part[threadIdx.x >> 6][a] = mn[a];
      part[threadIdx.x >> 6][3 + a] = mx[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    uint32_t v = part[0][a];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w)
      v = a < 3 ? min(v, part[w][a]) : max(v, part[w][a]);
    if (a < 3) atomicMin(&bbox_u[a], v);
    else atomicMax(&bbox_u[a], v);
  }
}

// hdr = {lo_x, lo_y, lo_z, L, 2^21 / L}.  L is the largest extent of the
// bounding box (1 if all elements coincide) unless the caller fixed a box.
__global__ void k_header(const uint32_t* bbox_u, double bx, double by, double bz, double bL,
                         double* hdr) {
  if (threadIdx.x != 0) return;
  double lo[3], L;
  if (bL > 0.0) {
    lo[0] = bx; lo[1] = by; lo[2] = bz; L = bL;
  } else {
    L = 0.0;
    for (int a = 0; a < 3; ++a) {
      lo[a] = (double)ord2f(bbox_u[a]);
      const double hi = (double)ord2f(bbox_u[3 + a]);
      L = fmax(L, hi - lo[a]);
    }
    if (L == 0.0) L = 1.0;
  }
  hdr[0] = lo[0]; hdr[1] = lo[1]; hdr[2] = lo[2]; hdr[3] = L;
  hdr[4] = ldexp(1.0, kKeyBits) / L;
}

// ----------------------------------------------------------- Morton keys
__global__ void k_keys(const float* x, const float* y, const float* z, const float* m,
                       const float* rho, const float* kappa, const float* lum, int64_t n,
                       int B, const double* hdr, uint64_t* keys, uint32_t* vals,
                       uint32_t* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float X[3] = {x[i], y[i], z[i]};
  bool ok = isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]) && finite_pos(m[i]) &&
            finite_pos(rho[i]);
  for (int b = 0; b < B; ++b) {
    const float kv = kappa[(int64_t)b * n + i], lv = lum[(int64_t)b * n + i];
    ok = ok && isfinite(kv) && kv >= 0.0f && isfinite(lv) && lv >= 0.0f;
  }
  if (!ok) atomicOr(err, ERR_DATA);
  uint32_t q[3];
  const double scale = hdr[4];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double u = floor(((double)X[a] - hdr[a]) * scale);
    if (!(u >= 0.0)) u = 0.0;
    if (u > 2097151.0) u = 2097151.0;
    q[a] = (uint32_t)u;
  }
  uint64_t k = 0;
  for (int b = kKeyBits - 1; b >= 0; --b)
#pragma unroll
    for (int a = 0; a < 3; ++a) k = (k << 1) | (uint64_t)((q[a] >> b) & 1u);
  keys[i] = k;
  vals[i] = (uint32_t)i;
}

// ------------------------------------------- stable LSD radix sort, 8 bits
__global__ void __launch_bounds__(256) k_sort_hist(const uint64_t* keys, int64_t n, int shift,
                                                   uint32_t* hist, int nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SortCfg::kTile;
  for (int r = 0; r < SortCfg::kItems; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(256) k_sort_scatter(const uint64_t* kin, const uint32_t* vin,
                                                      uint64_t* kout, uint32_t* vout,
                                                      int64_t n, int shift,
                                                      const uint32_t* hist, int nblk) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x, w = t >> 6;
  run[t] = 0u;
  goff[t] = hist[(int64_t)t * nblk + blockIdx.x];
  wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SortCfg::kTile;
  for (int r = 0; r < SortCfg::kItems; ++r) {
    const int64_t i = base + r * 256 + t;
    const bool valid = i < n;
    const uint64_t k = valid ? kin[i] : 0ull;
    const uint32_t v = valid ? vin[i] : 0u;
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t mm = ballot64(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = ballot64(on);
      mm &= on ? bb : ~bb;
    }
    const int rank_w = mbcnt(mm);
    if (valid && rank_w == 0) wcnt[w][d] = (uint32_t)__popcll(mm);
    __syncthreads();
    if (valid) {
      uint32_t pre = run[d];
      for (int ww = 0; ww < w; ++ww) pre += wcnt[ww][d];
      const uint32_t dst = goff[d] + pre + (uint32_t)rank_w;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0u;
    __syncthreads();
  }
}

// ------------------------------------------------- sorted element arrays
__global__ void k_gather(const float* x, const float* y, const float* z, const float* m,
                         const float* rho, const float* kappa, const float* lum, int64_t n,
                         int B, const uint32_t* vals, TreeBufs tb) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t i = vals[s];
  tb.perm[s] = i;
  tb.x[s] = x[i];
  tb.y[s] = y[i];
  tb.z[s] = z[i];
  const float mi = m[i], ri = rho[i];
  tb.m[s] = mi;
  tb.rho[s] = ri;
  tb.h[s] = cbrt((double)mi / (double)ri);   // element size, Section 2.1
  double lb = 0.0;
  for (int b = 0; b < B; ++b) {
    const float lv = lum[(int64_t)b * n + i];
    tb.kappa[(int64_t)b * n + s] = kappa[(int64_t)b * n + i];
    tb.lum[(int64_t)b * n + s] = lv;
    lb += (double)lv;
  }
  tb.lbol[s] = lb;
}

// ------------------------------------------------------------- topology
__global__ void k_root(TreeBufs tb, int64_t n) {
  if (threadIdx.x != 0) return;
  tb.b_first[0] = 0u;
  tb.b_count[0] = (uint32_t)n;
  tb.b_lown[0] = 0;
  tb.b_pre[0] = 0u;
  tb.levels[0] = make_uint2(0u, 1u);
}

// One level: a node is a bucket if it holds at most leaf_size elements or
// all its keys are equal; otherwise it splits at the first bit in which its
// keys differ (its sorted range splits where that bit turns on).
// The level's range [lb, le) is read from levels[d] (written by the previous
// level's k_level_next), so levels follow each other without the host.
__global__ void k_level(TreeBufs tb, int d, int leaf_size) {
  const uint2 lv = tb.levels[d];
  const uint32_t i = lv.x + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lv.y) return;
  const uint32_t f = tb.b_first[i], c = tb.b_count[i];
  const uint64_t k0 = tb.keys[f], k1 = tb.keys[f + c - 1];
  if (c <= (uint32_t)leaf_size || k0 == k1) {
    tb.b_split[i] = -1;
    return;
  }
  const int s = __clzll((long long)(k0 ^ k1)) - 1;
  const uint64_t bit = 1ull << (62 - s);
  uint32_t lo = f, hi = f + c - 1;  // key[lo] lacks the bit, key[hi] has it
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (tb.keys[mid] & bit) hi = mid; else lo = mid;
  }
  const uint32_t pos = atomicAdd(tb.alloc, 2u);
  tb.b_first[pos] = f;
  tb.b_count[pos] = hi - f;
  tb.b_lown[pos] = s + 1;
  tb.b_first[pos + 1] = hi;
  tb.b_count[pos + 1] = f + c - hi;
  tb.b_lown[pos + 1] = s + 1;
  tb.b_c0[i] = pos;
  tb.b_c1[i] = pos + 1;
  tb.b_split[i] = s;
}

// Range of level d + 1: the nodes allocated by the splits of level d.
__global__ void k_level_next(TreeBufs tb, int d) {
  if (threadIdx.x == 0) tb.levels[d + 1] = make_uint2(tb.levels[d].y, *tb.alloc);
}

__global__ void k_sizes(TreeBufs tb, uint32_t lb, uint32_t le) {
  const uint32_t i = lb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= le) return;
  tb.b_size[i] = (tb.b_split[i] < 0) ? 1u : 1u + tb.b_size[tb.b_c0[i]] + tb.b_size[tb.b_c1[i]];
}

__global__ void k_preorder(TreeBufs tb, uint32_t lb, uint32_t le) {
  const uint32_t i = lb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= le || tb.b_split[i] < 0) return;
  const uint32_t p = tb.b_pre[i];
  const uint32_t c0 = tb.b_c0[i];
  tb.b_pre[c0] = p + 1u;
  tb.b_pre[tb.b_c1[i]] = p + 1u + tb.b_size[c0];
}

__device__ inline uint32_t compact3(uint64_t k, int a) {
  // bits of axis a sit at positions 3b + (2 - a)
  uint32_t q = 0;
  for (int b = 0; b < kKeyBits; ++b) q |= (uint32_t)((k >> (3 * b + 2 - a)) & 1ull) << b;
  return q;
}

__global__ void k_scatter_nodes(TreeBufs tb, uint32_t total) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint32_t p = tb.b_pre[i];
  const int l = tb.b_lown[i];
  const uint64_t key = tb.keys[tb.b_first[i]];
  uint32_t kk[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) kk[a] = compact3(key, a) >> (kKeyBits - nbits_axis(l, a));
  const bool leaf = tb.b_split[i] < 0;
  tb.nk[p] = make_uint4(kk[0], kk[1], kk[2], (uint32_t)l | (leaf ? META_LEAF : 0u));
  tb.nlink[p] = leaf ? make_uint2(tb.b_first[i], tb.b_count[i])
                     : make_uint2(tb.b_pre[tb.b_c1[i]], (uint32_t)tb.b_split[i]);
  tb.next[p] = p + tb.b_size[i];
}

// --------------------------------------------------------------- moments
// Bucket sums over the elements in key order, parents as child0 + child1.
// The bucket absorption is sum(kappa m) / sum(m / rho) (Section 2.6);
// the centre of luminosity is sum(Lbol x)/Lbol, the box centre when dark.
__global__ void k_moments(TreeBufs tb, uint32_t lb, uint32_t le, int64_t n, int B, int nclass) {
  const uint32_t i = lb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= le) return;
  const uint32_t p = tb.b_pre[i];
  double Lb[kMaxBands], sl[3] = {0.0, 0.0, 0.0}, lbol = 0.0, kmass = 0.0;
  for (int b = 0; b < B; ++b) Lb[b] = 0.0;
  uint4 nk = tb.nk[p];
  if (tb.b_split[i] < 0) {
    double kmv[kMaxBands], vol = 0.0;
    for (int b = 0; b < B; ++b) kmv[b] = 0.0;
    const uint32_t f = tb.b_first[i], c = tb.b_count[i];
    for (uint32_t s = f; s < f + c; ++s) {
      const double ms = (double)tb.m[s];
      for (int b = 0; b < B; ++b) {
        const double kv = (double)tb.kappa[(int64_t)b * n + s];
        Lb[b] += (double)tb.lum[(int64_t)b * n + s];
        kmv[b] += kv * ms;
        kmass += kv * ms;
      }
      const double lbs = tb.lbol[s];
      lbol += lbs;
      sl[0] += lbs * (double)tb.x[s];
      sl[1] += lbs * (double)tb.y[s];
      sl[2] += lbs * (double)tb.z[s];
      vol += ms / (double)tb.rho[s];
    }
    const int64_t row = (int64_t)p * nclass * B;
    for (int b = 0; b < B; ++b) {
      const double ab = kmv[b] / vol;
      for (int c2 = 0; c2 < nclass; ++c2) {
        tb.alpha64[row + (int64_t)c2 * B + b] = ab;
        tb.alpha32[row + (int64_t)c2 * B + b] = (float)ab;
      }
    }
  } else {
    const uint32_t p0 = p + 1u, p1 = tb.nlink[p].x;
    for (int b = 0; b < B; ++b)
      Lb[b] = tb.Lb[(int64_t)p0 * B + b] + tb.Lb[(int64_t)p1 * B + b];
    const double4 s0 = tb.sl[p0], s1 = tb.sl[p1];
    lbol = s0.w + s1.w;
    sl[0] = s0.x + s1.x;
    sl[1] = s0.y + s1.y;
    sl[2] = s0.z + s1.z;
    kmass = tb.kmass[p0] + tb.kmass[p1];
  }
  for (int b = 0; b < B; ++b) tb.Lb[(int64_t)p * B + b] = Lb[b];
  tb.sl[p] = make_double4(sl[0], sl[1], sl[2], lbol);
  tb.kmass[p] = kmass;
  double lo[3], hi[3];
  node_box(tb.hdr, nk, lo, hi);
  double c[3];
  for (int a = 0; a < 3; ++a) c[a] = (lbol > 0.0) ? sl[a] / lbol : 0.5 * (lo[a] + hi[a]);
  tb.cen[p] = make_double4(c[0], c[1], c[2], lbol);
  nk.w |= (lbol > 0.0 ? META_LUM : 0u) | (kmass > 0.0 ? META_ABS : 0u);
  tb.nk[p] = nk;
}

// Internal nodes of one level, one thread per (node, direction class): the
// two children combine on the split box, then the result grows through the
// empty prefix boxes up to the owned box (empty space is vacuum).  With
// `linear` (TREVR_ABSORPTION_AVG) the combine is the linear volume-weighted
// mean instead of the transmission average.
__global__ void k_alpha(TreeBufs tb, uint32_t lb, uint32_t le, int B, int nclass, int linear) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t cnt = (int64_t)(le - lb) * nclass;
  if (gid >= cnt) return;
  const uint32_t i = lb + (uint32_t)(gid / nclass);
  const int c = (int)(gid % nclass);
  const int s = tb.b_split[i];
  if (s < 0) return;
  const uint32_t p = tb.b_pre[i], p0 = p + 1u, p1 = tb.nlink[p].x;
  const int l = tb.b_lown[i];
  const double L = tb.hdr[3];
  for (int b = 0; b < B; ++b) {
    const double a1 = tb.alpha64[((int64_t)p0 * nclass + c) * B + b];
    const double a2 = tb.alpha64[((int64_t)p1 * nclass + c) * B + b];
    double A;
    if (linear) {
      A = combine_linear(a1, a2);
      for (int mm = s - 1; mm >= l; --mm) A = combine_linear(A, 0.0);
    } else {
      A = combine64(&tb.geom[((int64_t)s * nclass + c) * 3], L, a1, a2);
      for (int mm = s - 1; mm >= l; --mm)
        A = combine64(&tb.geom[((int64_t)mm * nclass + c) * 3], L, A, 0.0);
    }
    tb.alpha64[((int64_t)p * nclass + c) * B + b] = A;
    tb.alpha32[((int64_t)p * nclass + c) * B + b] = (float)A;
  }
}

// Complex source model (Section 2.7, eq. srccomb, Fig. sourcecombine): the
// nodes of one level, one thread per (node, direction k over all N_ray).
// The ray from the node's luminosity centre c along n_k runs to the edge of
// the node's box (length d).  A bucket's ray sees the bucket absorption.  A
// merged node brings its children's rays to the same projected stopping
// point, the plane through c + d n_k normal to n_k: child i needs length
// D_i = d + (c - c_i).n_k, of which its own ray covers up to d_i (clipped
// when shorter, nothing when D_i <= 0) and the rest crosses the node with
// its transmission-averaged absorption in direction k; the optical depths
// combine so that attenuated luminosities add, per band:
//   L e^{-tau} = L_1 e^{-tau_1} + L_2 e^{-tau_2},
// and the node keeps alpha = tau / d (zero when d = 0 or L = 0).  Runs after
// k_alpha of the same level (it reads the node's transmission averages).
__global__ void k_csrc(TreeBufs tb, uint32_t lb, uint32_t le, int B, int nclass, int nray) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)(le - lb) * nray) return;
  const uint32_t i = lb + (uint32_t)(gid / nray);
  const int k = (int)(gid % nray);
  const uint32_t p = tb.b_pre[i];
  const double4 cp = tb.cen[p];
  const double c[3] = {cp.x, cp.y, cp.z};
  double lo[3], hi[3];
  node_box(tb.hdr, tb.nk[p], lo, hi);
  const double* nv = &tb.ray_n[3 * k];
  double dn = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (nv[a] > 0.0) dn = fmin(dn, (hi[a] - c[a]) / nv[a]);
    else if (nv[a] < 0.0) dn = fmin(dn, (lo[a] - c[a]) / nv[a]);
  }
  dn = fmax(dn, 0.0);
  tb.csrc_d[(int64_t)p * nray + k] = dn;
  double* out = &tb.csrc_a[((int64_t)p * nray + k) * B];
  if (tb.b_split[i] < 0) {
    for (int b = 0; b < B; ++b) out[b] = tb.alpha64[(int64_t)p * nclass * B + b];
    return;
  }
  const uint32_t ch[2] = {p + 1u, tb.nlink[p].x};
  double Dq[2], dq[2];
  for (int q = 0; q < 2; ++q) {
    const double4 cc = tb.cen[ch[q]];
    double D = dn;
    D += (c[0] - cc.x) * nv[0];
    D += (c[1] - cc.y) * nv[1];
    D += (c[2] - cc.z) * nv[2];
    Dq[q] = D;
    dq[q] = tb.csrc_d[(int64_t)ch[q] * nray + k];
  }
  const int cls = tb.ray_class[k];
  for (int b = 0; b < B; ++b) {
    const double Ln = tb.Lb[(int64_t)p * B + b];
    double al = 0.0;
    if (Ln > 0.0 && dn > 0.0) {
      const double aext = tb.alpha64[((int64_t)p * nclass + cls) * B + b];
      double tau[2], w[2];
      for (int q = 0; q < 2; ++q) {
        w[q] = tb.Lb[(int64_t)ch[q] * B + b] / Ln;
        const double ai = tb.csrc_a[((int64_t)ch[q] * nray + k) * B + b];
        if (!(Dq[q] > 0.0)) tau[q] = 0.0;
        else if (Dq[q] <= dq[q]) tau[q] = ai * Dq[q];
        else tau[q] = ai * dq[q] + aext * (Dq[q] - dq[q]);
      }
      int first = -1;
      for (int q = 0; q < 2; ++q)
        if (w[q] > 0.0 && (first < 0 || tau[q] < tau[first])) first = q;
      double sum = 0.0;
      for (int q = 0; q < 2; ++q)
        if (w[q] > 0.0) sum += w[q] * exp(-(tau[q] - tau[first]));
      al = (tau[first] - log(sum)) / dn;
    }
    out[b] = al;
  }
}

// ======================================================== host side
static void healpix_centres(int N, std::vector<double>& v) {
  v.assign(3 * 12 * N * N, 0.0);
  int k = 0;
  for (int i = 1; i <= 4 * N - 1; ++i) {
    double z, dphi, phi0;
    int cnt;
    if (i < N) {
      z = 1.0 - (double)i * i / (3.0 * N * N);
      cnt = 4 * i;
      dphi = kPi / (2.0 * i);
      phi0 = 0.5 * dphi;
    } else if (i <= 3 * N) {
      z = 4.0 / 3.0 - 2.0 * i / (3.0 * N);
      cnt = 4 * N;
      dphi = kPi / (2.0 * N);
      phi0 = ((i - N) % 2 == 0) ? 0.5 * dphi : 0.0;
    } else {
      const int ii = 4 * N - i;
      z = -(1.0 - (double)ii * ii / (3.0 * N * N));
      cnt = 4 * ii;
      dphi = kPi / (2.0 * ii);
      phi0 = 0.5 * dphi;
    }
    const double st = std::sqrt((1.0 - z) * (1.0 + z));
    for (int j = 0; j < cnt; ++j, ++k) {
      const double phi = phi0 + j * dphi;
      v[3 * k] = st * std::cos(phi);
      v[3 * k + 1] = st * std::sin(phi);
      v[3 * k + 2] = z;
    }
  }
}

// Ray-volume weights and chord of a box of sides s split across axis a,
// for lines along n (Section 2.6): V12 is the volume of lines crossing the
// joining face, V1 = V2 = (V - V12)/2, d the chord through the centre.
static void combine_geometry(const double s[3], int a, const double n[3], double out[3]) {
  const double V = s[0] * s[1] * s[2];
  double V12 = 0.0;
  if (n[a] != 0.0) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double tb = std::fabs(n[b] / n[a]), tc = std::fabs(n[c] / n[a]);
    double U = 0.5 * s[a];
    if (tb > 0.0) U = std::min(U, s[b] / tb);
    if (tc > 0.0) U = std::min(U, s[c] / tc);
    V12 = 2.0 * (s[b] * s[c] * U - (s[b] * tc + s[c] * tb) * U * U / 2.0 + tb * tc * U * U * U / 3.0);
  }
  const double w1 = std::max(0.0, (V - V12) / 2.0) / V;
  const double w12 = std::min(1.0, V12 / V);
  double d = INFINITY;
  for (int c = 0; c < 3; ++c)
    if (n[c] != 0.0) d = std::min(d, s[c] / std::fabs(n[c]));
  out[0] = (w1 > 0.0) ? std::log(w1) : -INFINITY;
  out[1] = (w12 > 0.0) ? std::log(w12) : -INFINITY;
  out[2] = d;
}

DirTables make_dir_tables(int nside) {
  DirTables t;
  t.nside = nside;
  t.nray = 12 * nside * nside;
  healpix_centres(nside, t.ray_n);
  t.ray_class.assign(t.nray, -1);
  std::vector<int> rep;
  for (int k = 0; k < t.nray; ++k) {
    const double* v = &t.ray_n[3 * k];
    int found = -1;
    for (size_t c = 0; c < rep.size() && found < 0; ++c) {
      const double* w = &t.ray_n[3 * rep[c]];
      if (std::fabs(std::fabs(v[0]) - std::fabs(w[0])) < 1e-12 &&
          std::fabs(std::fabs(v[1]) - std::fabs(w[1])) < 1e-12 &&
          std::fabs(std::fabs(v[2]) - std::fabs(w[2])) < 1e-12)
        found = (int)c;
    }
    if (found < 0) {
      found = (int)rep.size();
      rep.push_back(k);
    }
    t.ray_class[k] = found;
  }
  t.nclass = (int)rep.size();
  // antipodes: HEALPix centres come in opposite pairs, so -n_k is the centre
  // nearest to it
  t.ray_anti.assign(t.nray, 0);
  for (int k = 0; k < t.nray; ++k) {
    double best = INFINITY;
    for (int j = 0; j < t.nray; ++j) {
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double u = t.ray_n[3 * j + a] + t.ray_n[3 * k + a];
        d2 += u * u;
      }
      if (d2 < best) { best = d2; t.ray_anti[k] = j; }
    }
  }
  t.geom.assign((size_t)kMaxLevels * t.nclass * 3, 0.0);
  for (int l = 0; l < kMaxLevels; ++l) {
    double s[3];
    for (int a = 0; a < 3; ++a) s[a] = std::ldexp(1.0, -nbits_axis(l, a));
    for (int c = 0; c < t.nclass; ++c)
      combine_geometry(s, l % 3, &t.ray_n[3 * rep[c]], &t.geom[((size_t)l * t.nclass + c) * 3]);
  }
  return t;
}

size_t layout_tree(const trevr_params& p, int64_t n, int nclass, void* base, TreeBufs* o) {
  Carve cv(base);
  TreeBufs t{};
  const int64_t M = 2 * n;
  const int B = p.n_bands;
  const int nray = 12 * p.nside * p.nside;
  const int64_t nblk = (n + SortCfg::kTile - 1) / SortCfg::kTile;
  t.hdr = cv.take<double>(8);
  t.bbox_u = cv.take<uint32_t>(8);
  t.err = cv.take<uint32_t>(4);
  t.counters = cv.take<unsigned long long>(CNT_N);
  t.alloc = cv.take<uint32_t>(4);
  t.keys = cv.take<uint64_t>(n);
  t.keys_alt = cv.take<uint64_t>(n);
  t.vals = cv.take<uint32_t>(n);
  t.vals_alt = cv.take<uint32_t>(n);
  t.hist = cv.take<uint32_t>(256 * nblk + 1);
  t.x = cv.take<float>(n);
  t.y = cv.take<float>(n);
  t.z = cv.take<float>(n);
  t.m = cv.take<float>(n);
  t.rho = cv.take<float>(n);
  t.kappa = cv.take<float>(B * n);
  t.lum = cv.take<float>(B * n);
  t.h = cv.take<double>(n);
  t.lbol = cv.take<double>(n);
  t.perm = cv.take<uint32_t>(n);
  t.b_first = cv.take<uint32_t>(M);
  t.b_count = cv.take<uint32_t>(M);
  t.b_c0 = cv.take<uint32_t>(M);
  t.b_c1 = cv.take<uint32_t>(M);
  t.b_size = cv.take<uint32_t>(M);
  t.b_pre = cv.take<uint32_t>(M);
  t.b_lown = cv.take<int32_t>(M);
  t.b_split = cv.take<int32_t>(M);
  t.nk = cv.take<uint4>(M);
  t.nlink = cv.take<uint2>(M);
  t.next = cv.take<uint32_t>(M);
  t.cen = cv.take<double4>(M);
  t.sl = cv.take<double4>(M);
  t.Lb = cv.take<double>(M * B);
  t.kmass = cv.take<double>(M);
  t.alpha64 = cv.take<double>(M * nclass * B);
  t.alpha32 = cv.take<float>(M * nclass * B);
  t.ray_n = cv.take<double>(3 * nray);
  t.ray_class = cv.take<int32_t>(nray);
  t.ray_anti = cv.take<int32_t>(nray);
  t.csrc_d = nullptr;
  t.csrc_a = nullptr;
  if (p.flags & TREVR_COMPLEX_SRC) {
    t.csrc_d = cv.take<double>(M * nray);
    t.csrc_a = cv.take<double>(M * nray * B);
  }
  t.geom = cv.take<double>((size_t)kMaxLevels * nclass * 3);
  t.dev = cv.take<DevTree>(1);
  t.levels = cv.take<uint2>(kMaxLevels + 3);
  if (o) *o = t;
  return cv.off + 256;
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

trevr_status build_tree_impl(trevr_tree* T, const float* x, const float* y, const float* z,
                             const float* m, const float* rho, const float* kappa,
                             const float* lum) {
  const int64_t n = T->n;
  const int B = T->B;
  const int nclass = T->nclass;
  TreeBufs& tb = T->buf;
  hipStream_t st = T->stream;
  trevr_status rc;
#define TREVR_LAUNCH_CHECK(what)                                               \
  do {                                                                         \
    if ((rc = hip_check(hipGetLastError(), what)) != TREVR_OK) return rc;      \
  } while (0)

  // direction tables
  if ((rc = hip_check(hipMemcpyAsync(tb.ray_n, T->dirs.ray_n.data(),
                                     sizeof(double) * T->dirs.ray_n.size(),
                                     hipMemcpyHostToDevice, st), "copy rays")) != TREVR_OK) return rc;
  if ((rc = hip_check(hipMemcpyAsync(tb.ray_class, T->dirs.ray_class.data(),
                                     sizeof(int32_t) * T->dirs.ray_class.size(),
                                     hipMemcpyHostToDevice, st), "copy classes")) != TREVR_OK) return rc;
  if ((rc = hip_check(hipMemcpyAsync(tb.ray_anti, T->dirs.ray_anti.data(),
                                     sizeof(int32_t) * T->dirs.ray_anti.size(),
                                     hipMemcpyHostToDevice, st), "copy antipodes")) != TREVR_OK)
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(tb.geom, T->dirs.geom.data(),
                                     sizeof(double) * T->dirs.geom.size(),
                                     hipMemcpyHostToDevice, st), "copy geometry")) != TREVR_OK) return rc;

  k_init<<<1, 64, 0, st>>>(tb.bbox_u, tb.err, tb.counters, tb.alloc);
  TREVR_LAUNCH_CHECK("k_init");
  if (!(T->p.box[3] > 0.0)) {
    k_bbox<<<std::min<int64_t>(64, grid_for(n, 256)), 256, 0, st>>>(x, y, z, n, tb.bbox_u);
    TREVR_LAUNCH_CHECK("k_bbox");
  }
  k_header<<<1, 64, 0, st>>>(tb.bbox_u, T->p.box[0], T->p.box[1], T->p.box[2], T->p.box[3],
                             tb.hdr);
  TREVR_LAUNCH_CHECK("k_header");
  k_keys<<<grid_for(n, 256), 256, 0, st>>>(x, y, z, m, rho, kappa, lum, n, B, tb.hdr, tb.keys,
                                           tb.vals, tb.err);
  TREVR_LAUNCH_CHECK("k_keys");

  // radix sort: 8 passes of 8 bits, ping-pong ending in keys/vals
  const int nblk = (int)((n + SortCfg::kTile - 1) / SortCfg::kTile);
  uint64_t *ka = tb.keys, *kb = tb.keys_alt;
  uint32_t *va = tb.vals, *vb = tb.vals_alt;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    k_sort_hist<<<nblk, 256, 0, st>>>(ka, n, shift, tb.hist, nblk);
    TREVR_LAUNCH_CHECK("k_sort_hist");
    k_scan_u32<<<1, 1024, 0, st>>>(tb.hist, (int64_t)256 * nblk, nullptr);
    TREVR_LAUNCH_CHECK("k_scan_u32");
    k_sort_scatter<<<nblk, 256, 0, st>>>(ka, va, kb, vb, n, shift, tb.hist, nblk);
    TREVR_LAUNCH_CHECK("k_sort_scatter");
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  k_gather<<<grid_for(n, 256), 256, 0, st>>>(x, y, z, m, rho, kappa, lum, n, B, tb.vals, tb);
  TREVR_LAUNCH_CHECK("k_gather");

  // topology, top-down by level
  k_root<<<1, 64, 0, st>>>(tb, n);
  TREVR_LAUNCH_CHECK("k_root");
  // levels in batches, each level's range on the device; the host reads the
  // ranges back once per batch.  A level has at most twice the nodes of the
  // one above, which sizes the grids from the last width read back.
  T->levels.clear();
  constexpr int kLevelBatch = 6;
  uint64_t width = 1;   // nodes of level d
  int d = 0;
  for (bool done = false; !done;) {
    const int nb = std::min(kLevelBatch, kMaxLevels + 2 - d);
    if (nb <= 0) return set_error(TREVR_E_DATA, "tree deeper than the key allows");
    uint64_t bound = width;
    for (int k = 0; k < nb; ++k) {
      k_level<<<grid_for((int64_t)bound, 256), 256, 0, st>>>(tb, d + k, T->p.leaf_size);
      TREVR_LAUNCH_CHECK("k_level");
      k_level_next<<<1, 64, 0, st>>>(tb, d + k);
      TREVR_LAUNCH_CHECK("k_level_next");
      bound = std::min<uint64_t>(2 * bound, 2 * (uint64_t)n);
    }
    uint2* rb = reinterpret_cast<uint2*>(T->host_u32);   // levels d .. d + nb
    hipError_t e = hipMemcpyAsync(rb, tb.levels + d, sizeof(uint2) * (nb + 1),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if ((rc = hip_check(e, "level readback")) != TREVR_OK) return rc;
    for (int k = 0; k <= nb && !done; ++k) {
      if (rb[k].x >= rb[k].y) done = true;
      else if (k < nb) T->levels.emplace_back(rb[k].x, rb[k].y);
    }
    if (!done) width = rb[nb].y - rb[nb].x;
    d += nb;
  }
  if (T->levels.size() > (size_t)kMaxLevels + 2)
    return set_error(TREVR_E_DATA, "tree deeper than the key allows");
  const uint32_t total = T->levels.back().second;
  T->num_nodes = total;
  T->num_leaves = (total + 1) / 2;
  T->depth = (int32_t)T->levels.size();
  for (int d = T->depth - 1; d >= 0; --d) {
    const auto lv = T->levels[d];
    k_sizes<<<grid_for(lv.second - lv.first, 256), 256, 0, st>>>(tb, lv.first, lv.second);
    TREVR_LAUNCH_CHECK("k_sizes");
  }
  for (int d = 0; d < T->depth; ++d) {
    const auto lv = T->levels[d];
    k_preorder<<<grid_for(lv.second - lv.first, 256), 256, 0, st>>>(tb, lv.first, lv.second);
    TREVR_LAUNCH_CHECK("k_preorder");
  }
  k_scatter_nodes<<<grid_for(total, 256), 256, 0, st>>>(tb, total);
  TREVR_LAUNCH_CHECK("k_scatter_nodes");
  for (int d = T->depth - 1; d >= 0; --d) {
    const auto lv = T->levels[d];
    k_moments<<<grid_for(lv.second - lv.first, 128), 128, 0, st>>>(tb, lv.first, lv.second, n, B,
                                                                   nclass);
    TREVR_LAUNCH_CHECK("k_moments");
    const int64_t work = (int64_t)(lv.second - lv.first) * nclass;
    k_alpha<<<grid_for(work, 128), 128, 0, st>>>(tb, lv.first, lv.second, B, nclass,
                                                  (T->p.flags & TREVR_ABSORPTION_AVG) ? 1 : 0);
    TREVR_LAUNCH_CHECK("k_alpha");
    if (T->p.flags & TREVR_COMPLEX_SRC) {
      const int64_t cw = (int64_t)(lv.second - lv.first) * T->nray;
      k_csrc<<<grid_for(cw, 128), 128, 0, st>>>(tb, lv.first, lv.second, B, nclass, T->nray);
      TREVR_LAUNCH_CHECK("k_csrc");
    }
  }
#undef TREVR_LAUNCH_CHECK
  return TREVR_OK;
}

}  // namespace trevr
