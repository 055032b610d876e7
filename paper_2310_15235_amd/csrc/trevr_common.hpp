// Shared definitions of the MI355X TREVR2 library (device and host side).
// Method: Wadsley, Baumschlager & Shen (2023), "TREVR2" (MNRAS).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "trevr2.h"

namespace trevr {

constexpr int kMaxBands = 16;
constexpr int kMaxNside = 16;   // 3072 rays (pixel ids keep 16 bits in cut entries)
constexpr int kKeyBits = 21;           // bits per axis of the Morton key
constexpr int kMaxLevels = 64;         // prefix lengths 0..63
constexpr double kPi = 3.14159265358979323846;

// Sticky device error bits.
enum : uint32_t {
  ERR_DATA = 1u,         // non-positive or non-finite element data
  // (buffer overflows of a compute are handled by the host, which reruns
  // the affected step with more room: see OVF_* and walk_batch)
};

// Node meta word (nk.w): owned prefix length in bits 0..5, flags above.
enum : uint32_t {
  META_LEAF = 1u << 8,
  META_LUM = 1u << 9,     // bolometric luminosity > 0
  META_ABS = 1u << 10,    // sum of kappa*m > 0
};

// Cut list entry: id (node or sorted slot) and a meta word: pixel in bits
// 0..15 (0xFFFF = no source), kind in bits 16..17, absorbing flag bit 18.
enum : uint32_t {
  CUT_NOPIX = 0xFFFFu,
  CUT_CELL = 0u << 16,        // accepted cell (absorber and/or merged source)
  CUT_LEAF = 1u << 16,        // opened bucket: absorber only
  CUT_PART = 2u << 16,        // element source resolved from an opened bucket
  CUT_KIND_MASK = 3u << 16,
  CUT_ABS = 1u << 18,
};

// Counter slots (uint64 on the device).
enum { CNT_BUCKETS = 0, CNT_CELLS, CNT_ABS, CNT_SRC, CNT_SEG, CNT_NEAR_PAIRS, CNT_MAX_NEAR,
       CNT_NODES, CNT_SRC_PAIRS, CNT_NS_TRIPLES, CNT_MAX_CUT, CNT_MAX_STACK, CNT_NS_HITS,
       CNT_PP_LOG, CNT_N = 16 };

// Device view of a tree (all pointers into the caller's tree workspace).
struct DevTree {
  int64_t n;
  int32_t B, nside, nray, nclass, leaf_size;
  uint32_t flags;
  double theta2, rpp_min, wbeam;
  double target[3];           // aim of the directed ray (TREVR_DIRECTED)
  int32_t stack_limit;        // entries of the small traversal stack in use
  int64_t num_nodes;
  const double* hdr;          // root lo[3], L, quantisation scale
  // sorted elements
  const float *x, *y, *z, *m, *rho;
  const double *h, *lbol;
  const float *kappa, *lum;   // [B][n]
  const uint32_t* perm;       // slot -> input index
  // nodes in preorder
  const uint4* nk;            // k_x, k_y, k_z, meta
  const uint2* nlink;         // leaf: (first, count); internal: (child1, split)
  const uint32_t* next;       // preorder index after the subtree
  const double4* cen;         // luminosity centre, bolometric luminosity
  const double* Lb;           // [node][B]
  const float* alpha;         // [node][nclass][B]
  const double* ray_n;        // [nray][3]
  const int32_t* ray_class;   // [nray]
  const int32_t* ray_anti;    // [nray] ray of the opposite direction
  const double* csrc_d;       // complex source model (TREVR_COMPLEX_SRC): [node][nray]
  const double* csrc_a;       //   lengths and [node][nray][B] absorption of the
                              //   rays from each node's luminosity centre
  uint32_t* err;              // sticky error bits
  unsigned long long* counters;
  // tables of the build that the adjoint reads
  const uint32_t* b_pre;      // BFS index -> preorder index
  const int32_t *b_lown, *b_split;
  const double* alpha64;      // [node][nclass][B]
  const double* geom;         // [64][nclass][3]
  const uint2* levels;        // [depth] BFS index ranges per depth
  int32_t depth;
  // offsets of this tree's blocks in arrays shared by the scenes of a
  // forest (all zero for a tree on its own)
  int32_t boff;               // bands: background intensities
  int64_t eoff;               // elements: active flags, density gradients
  int64_t joff;               // [B][n] blocks: J, its adjoint, L and kappa gradients
  int64_t noff;               // nodes: centre adjoints (4 per node)
  int64_t lboff;              // node x band: luminosity adjoints
  int64_t aoff;               // node x class x band: transmission adjoints
};

// ------------------------------------------------------------ geometry
// Bits of prefix length l on axis a (x gets the first bit).
__host__ __device__ inline int nbits_axis(int l, int a) { return (l + 2 - a) / 3; }

// Box of a node from its integer prefix coordinates k and prefix length l.
__device__ inline void node_box(const double* hdr, uint4 nk, double lo[3], double hi[3]) {
  const int l = (int)(nk.w & 63u);
  const uint32_t kk[3] = {nk.x, nk.y, nk.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double side = ldexp(hdr[3], -nbits_axis(l, a));
    lo[a] = hdr[a] + (double)kk[a] * side;
    hi[a] = hdr[a] + (double)(kk[a] + 1u) * side;
  }
}

__device__ inline double dist2_box(const double lo[3], const double hi[3], const double c[3]) {
  double dd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    dd[a] = (c[a] < lo[a]) ? lo[a] - c[a] : (c[a] > hi[a] ? c[a] - hi[a] : 0.0);
  return dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
}

__device__ inline double far2_box(const double lo[3], const double hi[3], const double c[3]) {
  double e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = lo[a] - c[a], w = hi[a] - c[a];
    e[a] = fmax(u * u, w * w);
  }
  return e[0] + e[1] + e[2];
}

__device__ inline double dist2_pt3(double ax, double ay, double az, const double c[3]) {
  const double d0 = ax - c[0], d1 = ay - c[1], d2 = az - c[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}

// Slab intersection of the ray c + t n with a box.
__device__ inline bool slab(const double lo[3], const double hi[3], const double c[3],
                            const double n[3], const double inv[3], double& tin, double& tout) {
  tin = -INFINITY;
  tout = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (n[a] != 0.0) {
      const double t1 = (lo[a] - c[a]) * inv[a];
      const double t2 = (hi[a] - c[a]) * inv[a];
      tin = fmax(tin, fmin(t1, t2));
      tout = fmin(tout, fmax(t1, t2));
    } else if (c[a] < lo[a] || c[a] > hi[a]) {
      return false;
    }
  }
  return tin < tout;
}

// HEALPix ring-scheme pixel containing direction v (Gorski et al. 2005).
__device__ inline int healpix_pixel(int N, double x, double y, double zz) {
  const double r = sqrt(x * x + y * y + zz * zz);
  const double z = zz / r;
  const double za = fabs(z);
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 2.0 * kPi;
  const double tt = phi / (0.5 * kPi);
  const int ncap = 2 * N * (N - 1);
  if (za <= 2.0 / 3.0) {
    const double t1 = N * (0.5 + tt);
    const double t2 = N * z * 0.75;
    const long jp = (long)floor(t1 - t2);
    const long jm = (long)floor(t1 + t2);
    const long ir = N + 1 + jp - jm;
    const long kshift = 1 - (ir & 1);
    long ip = (jp + jm - N + kshift + 1) / 2;
    ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
    return (int)(ncap + (ir - 1) * 4 * N + ip);
  }
  const double tp = tt - floor(tt);
  const double tmp = N * sqrt(3.0 * (1.0 - za));
  const long jp = (long)floor(tp * tmp);
  const long jm = (long)floor((1.0 - tp) * tmp);
  const long ir = jp + jm + 1;
  long ip = (long)floor(tt * ir);
  ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
  if (z > 0) return (int)(2 * ir * (ir - 1) + ip);
  return (int)(12 * N * N - 2 * ir * (ir + 1) + ip);
}

// Directed rays (TREVR_DIRECTED; Sections 3.4.1, 4): the ray of a bucket
// with centre c whose pixel holds the direction to T.target is aimed exactly
// at the target.  Returns that ray's index and its unit direction u, or -1
// when the flag is off or the target is the bucket centre.
__device__ inline int directed_ray(const DevTree& T, const double c[3], double u[3]) {
  if (!(T.flags & TREVR_DIRECTED)) return -1;
  const double v0 = T.target[0] - c[0], v1 = T.target[1] - c[1], v2 = T.target[2] - c[2];
  if (v0 == 0.0 && v1 == 0.0 && v2 == 0.0) return -1;
  const double d = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  u[0] = v0 / d;
  u[1] = v1 / d;
  u[2] = v2 / d;
  return healpix_pixel(T.nside, v0, v1, v2);
}

// Transmission average of two halves (Section 2.6, eq. transmissionavg):
// exp(-d alpha) = w1 e^{-d a1} + w1 e^{-d a2} + w12 e^{-d (a1 + a2)/2},
// with the through-both rays taking half their length in each child.
__device__ inline double combine64(const double* g, double L, double a1, double a2) {
  const double lw1 = g[0], lw12 = g[1], d = g[2] * L;
  double t[3];
  int nt = 0;
  if (lw1 > -INFINITY) { t[nt++] = lw1 - d * a1; t[nt++] = lw1 - d * a2; }
  if (lw12 > -INFINITY) t[nt++] = lw12 - d * (a1 + a2) / 2.0;
  double mx = t[0];
  for (int k = 1; k < nt; ++k) mx = fmax(mx, t[k]);
  double s = 0.0;
  for (int k = 0; k < nt; ++k) s += exp(t[k] - mx);
  return -(mx + log(s)) / d;
}

// Linear volume-weighted absorption average of two equal halves (Section
// 2.6, the scheme the transmission average replaces; TREVR_ABSORPTION_AVG).
// Its partial derivatives are 1/2 each.
__device__ inline double combine_linear(double a1, double a2) { return 0.5 * (a1 + a2); }

// combine64 and its partial derivatives with respect to a1 and a2: with
// softmax weights p_k of the three log-terms, d alpha/d a1 = p1 + p3/2 and
// d alpha/d a2 = p2 + p3/2 (the through-both rays see each half for half
// their length).
__device__ inline double combine64_d(const double* g, double L, double a1, double a2, double* d1,
                                     double* d2) {
  const double lw1 = g[0], lw12 = g[1], d = g[2] * L;
  const bool h1 = lw1 > -INFINITY, h12 = lw12 > -INFINITY;
  const double t1 = h1 ? lw1 - d * a1 : -INFINITY;
  const double t2 = h1 ? lw1 - d * a2 : -INFINITY;
  const double t3 = h12 ? lw12 - d * (a1 + a2) / 2.0 : -INFINITY;
  const double mx = fmax(fmax(t1, t2), t3);
  const double e1 = h1 ? exp(t1 - mx) : 0.0, e2 = h1 ? exp(t2 - mx) : 0.0;
  const double e3 = h12 ? exp(t3 - mx) : 0.0;
  const double s = e1 + e2 + e3;
  *d1 = (e1 + 0.5 * e3) / s;
  *d2 = (e2 + 0.5 * e3) / s;
  return -(mx + log(s)) / d;
}

// ------------------------------------------------------------ wave helpers
__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }
__device__ inline int mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Exclusive scan of `total` uint32 in place by one workgroup of 1024
// threads, in chunks of 1024 x kScanPer words (each thread's kScanPer
// consecutive words loaded together, wavefront scans, then the 16 wavefront
// totals); the grand total goes to *sum_out when given.
constexpr int kScanPer = 16;
__device__ inline void block_scan_u32(uint32_t* a, int64_t total, uint32_t* sum_out) {
  __shared__ uint32_t wtot[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t carry = 0;
  for (int64_t base = 0; base < total; base += 1024 * kScanPer) {
    const int64_t i0 = base + (int64_t)t * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = (i0 + k < total) ? a[i0 + k] : 0u;
      s += v[k];
    }
    uint32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)incl, o);
      if (lane >= o) incl += u;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    uint32_t wbase = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const uint32_t x = wtot[w];
      if (w < wv) wbase += x;
      btot += x;
    }
    __syncthreads();
    uint32_t run = carry + wbase + (incl - s);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < total) a[i0 + k] = run;
      run += v[k];
    }
    carry += btot;
  }
  if (t == 0 && sum_out) *sum_out = carry;
}

static __global__ void __launch_bounds__(1024) k_scan_u32(uint32_t* a, int64_t total,
                                                          uint32_t* sum_out) {
  block_scan_u32(a, total, sum_out);
}

// Up to four arrays of `total` words scanned at once, one workgroup each.
struct ScanArrays {
  uint32_t* a[4];
};
static __global__ void __launch_bounds__(1024) k_scan_arrays(ScanArrays s, int64_t total) {
  block_scan_u32(s.a[blockIdx.x], total, nullptr);
}

}  // namespace trevr
