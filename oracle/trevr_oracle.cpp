// TREVR2 oracle: a plain, slow, FP64 CPU implementation of the radiative
// transfer method of Wadsley, Baumschlager & Shen (2023), "TREVR2: Illuminating
// fast N log2 N radiative transfer" (MNRAS).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call this
// library: only the test suite, the smoke check and the benchmark's CPU
// baseline leg use it.  It includes no header of, and is linked with nothing
// from, the HIP implementation.  The FP64 decisions below (Healpix::pixel and
// the centres, dist2_box, far2_box, open_cell, slab, combine_geom) use the
// same operation order as the HIP library's so that discrete decisions agree
// bit for bit; they are pinned by CPU tests that do not involve the HIP
// library (closed forms, brute force, the paper's printed values).
//
// Every function follows the paper's definitions step by step, with plain
// loops and recursion and no blocking or reordering beyond what the
// definition states.  Where the paper is silent or ambiguous the reading taken
// is stated next to the code.  The scalar type is a template parameter so the
// same code also yields exact forward-mode derivatives (dual numbers) with all
// discrete decisions taken on the values, i.e. frozen.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fPIC -shared
// (contraction is disabled so that every decision is a sequence of correctly
// rounded IEEE operations).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- scalars --
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); return Dual(e, a.d * e); }
inline Dual log(const Dual& a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d == 0.0 ? 0.0 : a.d / (2.0 * s));
}
inline Dual cbrt(const Dual& a) {
  double c = std::cbrt(a.v);
  return Dual(c, a.d / (3.0 * c * c));
}
inline Dual expm1(const Dual& a) { return Dual(std::expm1(a.v), a.d * std::exp(a.v)); }
inline Dual atanh(const Dual& a) { return Dual(std::atanh(a.v), a.d / (1.0 - a.v * a.v)); }

inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
inline double tan_(double) { return 0.0; }
inline double tan_(const Dual& a) { return a.d; }
using std::exp; using std::log; using std::sqrt; using std::cbrt; using std::expm1; using std::atanh;

// Larger of two scalars by value; ties keep the first argument.
template <class T> inline T vmax(const T& a, const T& b) { return val(b) > val(a) ? b : a; }

const double kPi = 3.14159265358979323846;

// ------------------------------------------------------------- parameters --
// Same field meaning as the library's parameter struct; declared here
// independently.
struct Params {
  int32_t nside;
  int32_t leaf_size;
  int32_t n_bands;
  uint32_t flags;
  double theta;
  double rpp_min;
  double box[4];
  double target[3];
};
enum : uint32_t { F_THICK = 1u, F_NEAR = 2u, F_BG = 4u, F_AVG = 8u, F_DIRECTED = 32u,
                  F_CPLX = 64u };

enum { C_BUCKETS = 0, C_CELLS, C_ABS, C_SRC, C_SEG, C_NEAR_PAIRS, C_MAX_NEAR, C_NODES,
       C_SRC_PAIRS, C_NS_TRIPLES, C_NS_HITS, C_N };

// ------------------------------------------------- element physics (2.1-2.4)
// Finite-element intensity kernel, Section 2.2, eq. (intint): the volume
// average over a uniform sphere of radius R h, R = (3/4pi)^(1/2), of the
// angle-integrated intensity of a unit point source at distance r.  Returned
// normalised so that L*K is the angle-integrated intensity (1/(4 pi r^2) far
// away, 1/h^2 at r = 0).  The logarithm of the paper's form is written with
// atanh: ln((x-1)^2/(x+1)^2) = -4 atanh(x) (x<1) or -4 atanh(1/x) (x>1).  For
// x >= 10 the cancellation is avoided with the series
// f = sum_k 2 x^(-2k) / (4k^2 - 1).
template <class T> T kernel_K(const T& r, const T& h) {
  const double R = std::sqrt(3.0 / (4.0 * kPi));
  T x = r / (R * h);
  double xv = val(x);
  T f;
  if (xv == 0.0) {
    f = T(2.0);
  } else if (xv < 1.0) {
    f = 1.0 + (1.0 - x * x) * atanh(x) / x;
  } else if (xv == 1.0) {
    f = T(1.0);
  } else if (xv < 10.0) {
    f = 1.0 - (x * x - 1.0) * atanh(1.0 / x) / x;
  } else {
    T y2 = 1.0 / (x * x);
    T term = y2;
    f = T(0.0);
    for (int k = 1; k < 60; ++k) {
      f += 2.0 * term / (4.0 * k * k - 1.0);
      term = term * y2;
      if (val(term) < 1e-22) break;
    }
  }
  return f / (2.0 * h * h);
}

// Optically thick element correction, Section 2.1, eq. (taucorr):
// <I> = I(0) (1 - e^-tau)/tau.
template <class T> T thick_C(const T& tau) {
  if (val(tau) == 0.0) return T(1.0);
  return -expm1(-tau) / tau;
}

// Particle column profile, Section 2.4: falls linearly with impact parameter b
// and integrates to the particle mass over the disc b < h.
template <class T> T column_sigma(double b, double m, const T& h) {
  return (3.0 * m / (kPi * h * h)) * (1.0 - b / h);
}

// ----------------------------------------------------------- HEALPix (1.3) --
// Ring-scheme pixel centres and point-in-pixel test of Gorski et al. (2005,
// ApJ 622, 759), N_ray = 12 nside^2 equal-area pixels.
struct Healpix {
  int nside, npix;
  std::vector<double> v;  // [npix][3] centres
  explicit Healpix(int ns) : nside(ns), npix(12 * ns * ns), v(3 * (size_t)npix) {
    const int N = ns;
    int k = 0;
    for (int i = 1; i <= 4 * N - 1; ++i) {
      double z, phi0, dphi;
      int cnt;
      if (i < N) {  // north polar cap
        z = 1.0 - (double)i * i / (3.0 * N * N);
        cnt = 4 * i;
        dphi = kPi / (2.0 * i);
        phi0 = 0.5 * dphi;
      } else if (i <= 3 * N) {  // equatorial belt
        z = 4.0 / 3.0 - 2.0 * i / (3.0 * N);
        cnt = 4 * N;
        dphi = kPi / (2.0 * N);
        phi0 = ((i - N) % 2 == 0) ? 0.5 * dphi : 0.0;
      } else {  // south polar cap
        int ii = 4 * N - i;
        z = -(1.0 - (double)ii * ii / (3.0 * N * N));
        cnt = 4 * ii;
        dphi = kPi / (2.0 * ii);
        phi0 = 0.5 * dphi;
      }
      double st = std::sqrt((1.0 - z) * (1.0 + z));
      for (int j = 0; j < cnt; ++j) {
        double phi = phi0 + j * dphi;
        v[3 * k + 0] = st * std::cos(phi);
        v[3 * k + 1] = st * std::sin(phi);
        v[3 * k + 2] = z;
        ++k;
      }
    }
  }
  // Pixel containing direction (x, y, z) (need not be normalised).
  int pixel(double x, double y, double zz) const {
    const int N = nside;
    double r = std::sqrt(x * x + y * y + zz * zz);
    double z = zz / r;
    double za = std::fabs(z);
    double phi = std::atan2(y, x);
    if (phi < 0.0) phi += 2.0 * kPi;
    double tt = phi / (0.5 * kPi);  // in [0, 4]
    const int ncap = 2 * N * (N - 1);
    if (za <= 2.0 / 3.0) {
      // Equatorial belt: pixel edges are straight lines in (phi, z).
      double t1 = N * (0.5 + tt);
      double t2 = N * z * 0.75;
      long jp = (long)std::floor(t1 - t2);  // index of ascending edge line
      long jm = (long)std::floor(t1 + t2);  // index of descending edge line
      long ir = N + 1 + jp - jm;            // ring counted from z = 2/3, 1..2N+1
      long kshift = 1 - (ir & 1);
      long ip = (jp + jm - N + kshift + 1) / 2;
      ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
      return (int)(ncap + (ir - 1) * 4 * N + ip);
    }
    // Polar caps.
    double tp = tt - std::floor(tt);
    double tmp = N * std::sqrt(3.0 * (1.0 - za));
    long jp = (long)std::floor(tp * tmp);
    long jm = (long)std::floor((1.0 - tp) * tmp);
    long ir = jp + jm + 1;  // ring counted from the nearest pole
    long ip = (long)std::floor(tt * ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0) return (int)(2 * ir * (ir - 1) + ip);
    return (int)(npix - 2 * ir * (ir + 1) + ip);
  }
};

// -------------------------------------------------- transmission averaging --
// Section 2.6, eq. (transmissionavg), with the ray-volume weights and the
// chord d taken as follows (the paper gives them in words only):
//  * the box (sides s[3]) is split in half along axis a;
//  * V12 is the volume swept by lines along n that cross the joining face
//    inside the box: at depth u from the face the cross-section is
//    (s_b - t_b u)(s_c - t_c u), t_c = |n_c/n_a|, integrated to
//    U = min(s_a/2, s_b/t_b, s_c/t_c) and doubled for both halves;
//  * V1 = V2 = (V - V12)/2 (each half holds rays that miss the face);
//  * d is the chord of the ray through the box centre (the face centre).
// The through-both term is the product e^{-d a1/2} e^{-d a2/2} (the printed
// sum exceeds one at zero opacity; the product reproduces the printed
// thinnest/thickest rows of the two-cell table).  Evaluated as a log-sum-exp.
struct CombineGeom {
  double w1, w12, d;  // V1/V (= V2/V), V12/V, chord
};
CombineGeom combine_geom(const double s[3], int a, const double n[3]) {
  double V = s[0] * s[1] * s[2];
  double V12 = 0.0;
  if (n[a] != 0.0) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double tb = std::fabs(n[b] / n[a]);
    double tc = std::fabs(n[c] / n[a]);
    double U = 0.5 * s[a];
    if (tb > 0.0) U = std::min(U, s[b] / tb);
    if (tc > 0.0) U = std::min(U, s[c] / tc);
    V12 = 2.0 * (s[b] * s[c] * U - (s[b] * tc + s[c] * tb) * U * U / 2.0 +
                 tb * tc * U * U * U / 3.0);
  }
  double V1 = std::max(0.0, (V - V12) / 2.0);
  double d = std::numeric_limits<double>::infinity();
  for (int c = 0; c < 3; ++c)
    if (n[c] != 0.0) d = std::min(d, s[c] / std::fabs(n[c]));
  CombineGeom g;
  g.w1 = V1 / V;
  g.w12 = std::min(1.0, V12 / V);
  g.d = d;
  return g;
}

template <class T> T combine_alpha(const CombineGeom& g, const T& a1, const T& a2) {
  T t[3] = {T(0.0), T(0.0), T(0.0)};
  int nt = 0;
  if (g.w1 > 0.0) {
    t[nt++] = std::log(g.w1) - g.d * a1;
    t[nt++] = std::log(g.w1) - g.d * a2;
  }
  if (g.w12 > 0.0) t[nt++] = std::log(g.w12) - g.d * (a1 + a2) / 2.0;
  T mx = t[0];
  for (int i = 1; i < nt; ++i) mx = vmax(mx, t[i]);
  T s = T(0.0);
  for (int i = 0; i < nt; ++i) s += exp(t[i] - mx);
  T lnT = mx + log(s);
  return -lnT / g.d;
}

// --------------------------------------------------------------- the tree --
// Section 2.3: binary tree, each division half-way along the longest axis,
// buckets of at most leaf_size particles.  Realised as a radix tree over
// 63-bit Morton keys (x bit first): a node covers a contiguous range of
// sorted particles; it is a leaf if it holds at most leaf_size particles or
// all its keys are equal, otherwise it is split at the first bit s in which
// its keys differ.  The node owns the prefix box of length (parent's s + 1);
// boxes of length l are split along axis l mod 3, so every box is a cube or
// 2:1 and the longest axis is always the one halved (ties x, y, z).
struct NodeG {
  int64_t first, count;
  int lown, split;  // owned prefix length; split bit (-1 for leaves)
  int64_t c0, c1, next;
  bool leaf;
  double lo[3], hi[3];
};

struct Tree {
  Params p;
  int64_t n;
  int B, nray, ndir;
  double lo[3], L;
  std::vector<int64_t> perm;  // sorted slot -> input index
  std::vector<uint64_t> key;  // sorted keys
  std::vector<uint32_t> q;    // [slot][3]
  std::vector<double> x;      // [slot][3]
  std::vector<double> m;      // [slot]
  std::vector<NodeG> node;    // depth-first preorder, child 0 first
  Healpix hp;
  std::vector<int> dir_of_ray;  // stored direction index of each ray
  std::vector<int> ray_of_dir;  // representative ray of each stored direction
  std::vector<int> antipode;    // ray of the opposite direction
  explicit Tree(int nside) : hp(nside) {}
};

inline int nbits_axis(int l, int a) { return (l + 2 - a) / 3; }

void prefix_box(const Tree& t, int64_t slot, int l, double lo[3], double hi[3]) {
  for (int a = 0; a < 3; ++a) {
    int nb = nbits_axis(l, a);
    double side = std::ldexp(t.L, -nb);
    uint32_t k = t.q[3 * slot + a] >> (21 - nb);
    lo[a] = t.lo[a] + (double)k * side;
    hi[a] = t.lo[a] + (double)(k + 1) * side;
  }
}

void box_sides(const Tree& t, int l, double s[3]) {
  for (int a = 0; a < 3; ++a) s[a] = std::ldexp(t.L, -nbits_axis(l, a));
}

int64_t build_node(Tree& t, int64_t f, int64_t c, int lown) {
  int64_t idx = (int64_t)t.node.size();
  t.node.push_back(NodeG());
  NodeG g;
  g.first = f;
  g.count = c;
  g.lown = lown;
  g.split = -1;
  g.c0 = g.c1 = -1;
  uint64_t k0 = t.key[f], k1 = t.key[f + c - 1];
  g.leaf = (c <= t.p.leaf_size) || (k0 == k1);
  prefix_box(t, f, lown, g.lo, g.hi);
  if (!g.leaf) {
    int s = __builtin_clzll(k0 ^ k1) - 1;  // first differing bit, 0 = x20
    uint64_t bit = 1ull << (62 - s);
    int64_t mid = f;
    while (!(t.key[mid] & bit)) ++mid;
    g.split = s;
    t.node[idx] = g;
    int64_t a = build_node(t, f, mid - f, s + 1);
    int64_t b = build_node(t, mid, f + c - mid, s + 1);
    g.c0 = a;
    g.c1 = b;
  }
  g.next = (int64_t)t.node.size();
  t.node[idx] = g;
  return idx;
}

Tree* build_geometry(const Params& p, int64_t n, const double* xs, const double* ys,
                     const double* zs, const double* ms) {
  Tree* t = new Tree(p.nside);
  t->p = p;
  t->n = n;
  t->B = p.n_bands;
  t->nray = 12 * p.nside * p.nside;
  const double* X[3] = {xs, ys, zs};
  // Root cube: the user box, else the bounding cube of the particles.
  if (p.box[3] > 0.0) {
    for (int a = 0; a < 3; ++a) t->lo[a] = p.box[a];
    t->L = p.box[3];
  } else {
    double hi[3];
    for (int a = 0; a < 3; ++a) {
      t->lo[a] = X[a][0];
      hi[a] = X[a][0];
      for (int64_t i = 1; i < n; ++i) {
        t->lo[a] = std::min(t->lo[a], X[a][i]);
        hi[a] = std::max(hi[a], X[a][i]);
      }
    }
    t->L = 0.0;
    for (int a = 0; a < 3; ++a) t->L = std::max(t->L, hi[a] - t->lo[a]);
    if (t->L == 0.0) t->L = 1.0;
  }
  // Quantise to 21 bits per axis and interleave, x first.
  const double scale = std::ldexp(1.0, 21) / t->L;
  std::vector<uint32_t> q(3 * (size_t)n);
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      double u = std::floor((X[a][i] - t->lo[a]) * scale);
      if (u < 0.0) u = 0.0;
      if (u > 2097151.0) u = 2097151.0;
      q[3 * i + a] = (uint32_t)u;
    }
    uint64_t k = 0;
    for (int b = 20; b >= 0; --b)
      for (int a = 0; a < 3; ++a) k = (k << 1) | ((q[3 * i + a] >> b) & 1u);
    key[i] = k;
  }
  // Sort by (key, input index).
  t->perm.resize(n);
  for (int64_t i = 0; i < n; ++i) t->perm[i] = i;
  std::sort(t->perm.begin(), t->perm.end(), [&](int64_t a, int64_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
  t->key.resize(n);
  t->q.resize(3 * (size_t)n);
  t->x.resize(3 * (size_t)n);
  t->m.resize(n);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t->perm[s];
    t->key[s] = key[i];
    for (int a = 0; a < 3; ++a) {
      t->q[3 * s + a] = q[3 * i + a];
      t->x[3 * s + a] = X[a][i];
    }
    t->m[s] = ms[i];
  }
  build_node(*t, 0, n, 0);
  // Stored directions: one per antipodal pair (Section 2.6: forward and
  // backward rays see the same average), keeping the lower pixel index.
  t->dir_of_ray.assign(t->nray, -1);
  for (int k = 0; k < t->nray; ++k) {
    const double* v = &t->hp.v[3 * k];
    int ka = t->hp.pixel(-v[0], -v[1], -v[2]);
    if (k < ka) {
      t->dir_of_ray[k] = (int)t->ray_of_dir.size();
      t->ray_of_dir.push_back(k);
    }
  }
  for (int k = 0; k < t->nray; ++k) {
    if (t->dir_of_ray[k] < 0) {
      const double* v = &t->hp.v[3 * k];
      int ka = t->hp.pixel(-v[0], -v[1], -v[2]);
      t->dir_of_ray[k] = t->dir_of_ray[ka];
    }
  }
  t->ndir = (int)t->ray_of_dir.size();
  t->antipode.resize(t->nray);
  for (int k = 0; k < t->nray; ++k) {
    const double* v = &t->hp.v[3 * k];
    t->antipode[k] = t->hp.pixel(-v[0], -v[1], -v[2]);
  }
  return t;
}

// Per-particle quantities in sorted order (Section 2.4, 2.6):
// h = (m/rho)^(1/3), bolometric luminosity = sum over bands.
template <class T> struct PartT {
  std::vector<T> rho, h, kappa, L, Lbol;  // kappa, L: [b][slot]
};

// Cell moments (Section 2.3, 2.6, Fig. sourcecombine): luminosities add and
// the combined source sits at the luminosity-weighted centre (one bolometric
// centre for all bands, so the traversal is band independent); buckets carry
// the volume-weighted absorption sum(kappa m)/sum(m/rho); larger cells the
// per-direction transmission average.  Sums are formed recursively, the
// children's sums added, leaves summing their particles in sorted order.
template <class T> struct Mom {
  std::vector<T> Lb, Lbol, SL, cen, alpha;  // Lb [node][B]; SL, cen [node][3]; alpha [node][ndir][B]
  std::vector<double> kmass;                // sum over particles and bands of kappa*m (value)
  // complex source model: per node and emission direction k (all N_ray), the
  // length of the ray from the luminosity centre to the edge of the node's
  // box and the absorption coefficient along it (per band)
  std::vector<T> cd, ca;                    // cd [node][nray]; ca [node][nray][B]
};

// Distance from c (inside the box) along n to the box's boundary.
template <class T> T exit_distance(const double lo[3], const double hi[3], const T c[3],
                                   const double n[3]) {
  T t = T(std::numeric_limits<double>::infinity());
  for (int a = 0; a < 3; ++a) {
    if (n[a] > 0.0) {
      T u = (hi[a] - c[a]) / n[a];
      if (val(u) < val(t)) t = u;
    } else if (n[a] < 0.0) {
      T u = (lo[a] - c[a]) / n[a];
      if (val(u) < val(t)) t = u;
    }
  }
  return vmax(t, T(0.0));
}

// Complex source model (Section 2.7, eq. srccomb, Fig. sourcecombine), built
// bottom-up after the transmission tables.  For node n and direction k the
// stored ray runs from the luminosity centre c_n along n_k to the edge of
// n's box (length d_n).  A bucket's ray sees the bucket absorption.  For a
// merged node the rays of the two children are brought to the same
// projected stopping point (the plane through c_n + d_n n_k normal to n_k):
// child i's ray needs length D_i = d_n + (c_n - c_i).n_k; its own segment
// covers up to d_i (clipped when D_i < d_i, none when D_i <= 0) and beyond it
// the ray crosses the rest of n with n's transmission-averaged absorption in
// direction k.  The optical depths combine so that the attenuated
// luminosities add: L_n e^{-tau_n} = L_1 e^{-tau_1} + L_2 e^{-tau_2}, and the
// node stores alpha_n = tau_n / d_n (zero when d_n = 0 or L_n = 0).
template <class T>
void complex_sources(const Tree& t, Mom<T>& mo) {
  const int64_t nn = (int64_t)t.node.size();
  const int B = t.B, K = t.nray, D = t.ndir;
  mo.cd.assign(nn * K, T(0.0));
  mo.ca.assign(nn * K * B, T(0.0));
  for (int64_t nd = nn - 1; nd >= 0; --nd) {
    const NodeG& g = t.node[nd];
    const T c[3] = {mo.cen[nd * 3 + 0], mo.cen[nd * 3 + 1], mo.cen[nd * 3 + 2]};
    for (int k = 0; k < K; ++k) {
      const double* n = &t.hp.v[3 * k];
      const T dn = exit_distance(g.lo, g.hi, c, n);
      mo.cd[nd * K + k] = dn;
      for (int b = 0; b < B; ++b) {
        T al = T(0.0);
        if (g.leaf) {
          al = mo.alpha[(nd * D + 0) * B + b];   // the bucket absorption, any direction
        } else if (val(mo.Lb[nd * B + b]) > 0.0 && val(dn) > 0.0) {
          const T aext = mo.alpha[(nd * D + t.dir_of_ray[k]) * B + b];
          T tau[2], w[2];
          const int64_t ch[2] = {g.c0, g.c1};
          for (int q = 0; q < 2; ++q) {
            const int64_t ci = ch[q];
            w[q] = mo.Lb[ci * B + b] / mo.Lb[nd * B + b];
            T Di = dn;
            for (int a = 0; a < 3; ++a) Di += (c[a] - mo.cen[ci * 3 + a]) * n[a];
            const T di = mo.cd[ci * K + k];
            const T ai = mo.ca[(ci * K + k) * B + b];
            if (!(val(Di) > 0.0)) {
              tau[q] = T(0.0);
            } else if (val(Di) <= val(di)) {
              tau[q] = ai * Di;
            } else {
              tau[q] = ai * di + aext * (Di - di);
            }
          }
          // -ln(w1 e^{-tau1} + w2 e^{-tau2}) about the smaller depth among
          // the luminous children
          int first = -1;
          for (int q = 0; q < 2; ++q)
            if (val(w[q]) > 0.0 && (first < 0 || val(tau[q]) < val(tau[first]))) first = q;
          T sum = T(0.0);
          for (int q = 0; q < 2; ++q)
            if (val(w[q]) > 0.0) sum += w[q] * exp(-(tau[q] - tau[first]));
          al = (tau[first] - log(sum)) / dn;
        }
        mo.ca[(nd * K + k) * B + b] = al;
      }
    }
  }
}

template <class T>
void compute_moments(const Tree& t, const PartT<T>& P, Mom<T>& mo) {
  const int64_t nn = (int64_t)t.node.size();
  const int B = t.B, D = t.ndir;
  mo.Lb.assign(nn * B, T(0.0));
  mo.Lbol.assign(nn, T(0.0));
  mo.SL.assign(nn * 3, T(0.0));
  mo.cen.assign(nn * 3, T(0.0));
  mo.alpha.assign(nn * D * B, T(0.0));
  mo.kmass.assign(nn, 0.0);
  // Children follow their parent in preorder, so a reverse sweep is bottom-up.
  for (int64_t nd = nn - 1; nd >= 0; --nd) {
    const NodeG& g = t.node[nd];
    if (g.leaf) {
      std::vector<T> kmv(B, T(0.0));
      T vol = T(0.0);
      for (int64_t s = g.first; s < g.first + g.count; ++s) {
        for (int b = 0; b < B; ++b) {
          mo.Lb[nd * B + b] += P.L[b * t.n + s];
          kmv[b] += P.kappa[b * t.n + s] * t.m[s];
          mo.kmass[nd] += val(P.kappa[b * t.n + s]) * t.m[s];
        }
        mo.Lbol[nd] += P.Lbol[s];
        for (int a = 0; a < 3; ++a) mo.SL[nd * 3 + a] += P.Lbol[s] * t.x[3 * s + a];
        vol += t.m[s] / P.rho[s];
      }
      for (int b = 0; b < B; ++b) {
        T ab = kmv[b] / vol;
        for (int j = 0; j < D; ++j) mo.alpha[(nd * D + j) * B + b] = ab;
      }
    } else {
      const int64_t a0 = g.c0, a1 = g.c1;
      for (int b = 0; b < B; ++b) mo.Lb[nd * B + b] = mo.Lb[a0 * B + b] + mo.Lb[a1 * B + b];
      mo.Lbol[nd] = mo.Lbol[a0] + mo.Lbol[a1];
      for (int a = 0; a < 3; ++a) mo.SL[nd * 3 + a] = mo.SL[a0 * 3 + a] + mo.SL[a1 * 3 + a];
      mo.kmass[nd] = mo.kmass[a0] + mo.kmass[a1];
      // Transmission average: combine the two children on the split box, then
      // grow through the empty prefix boxes up to the owned box (empty space
      // is vacuum).
      for (int j = 0; j < D; ++j) {
        const double* n = &t.hp.v[3 * t.ray_of_dir[j]];
        double s[3];
        box_sides(t, g.split, s);
        CombineGeom geo = combine_geom(s, g.split % 3, n);
        std::vector<CombineGeom> chain;
        for (int l = g.split - 1; l >= g.lown; --l) {
          box_sides(t, l, s);
          chain.push_back(combine_geom(s, l % 3, n));
        }
        for (int b = 0; b < B; ++b) {
          const T& al1 = mo.alpha[(a0 * D + j) * B + b];
          const T& al2 = mo.alpha[(a1 * D + j) * B + b];
          T A;
          if (t.p.flags & F_AVG) {
            // Linear absorption average (Section 2.6, the scheme transmission
            // averaging replaces): absorption coefficients weighted by volume.
            // The two children fill equal halves of the split box; every
            // empty prefix box above it doubles the volume with vacuum.
            A = (al1 + al2) / 2.0;
            for (size_t q = 0; q < chain.size(); ++q) A = A / 2.0;
          } else {
            A = combine_alpha(geo, al1, al2);
            for (const CombineGeom& cg : chain) A = combine_alpha(cg, A, T(0.0));
          }
          mo.alpha[(nd * D + j) * B + b] = A;
        }
      }
    }
    for (int a = 0; a < 3; ++a) {
      if (val(mo.Lbol[nd]) > 0.0)
        mo.cen[nd * 3 + a] = mo.SL[nd * 3 + a] / mo.Lbol[nd];
      else
        mo.cen[nd * 3 + a] = T(0.5 * (g.lo[a] + g.hi[a]));
    }
  }
}

template <class T>
void particle_props(const Tree& t, const double* rho, const double* kappa, const double* lum,
                    const double* trho, const double* tkappa, const double* tlum, PartT<T>& P);

template <>
void particle_props<double>(const Tree& t, const double* rho, const double* kappa, const double* lum,
                            const double*, const double*, const double*, PartT<double>& P) {
  const int64_t n = t.n;
  const int B = t.B;
  P.rho.resize(n); P.h.resize(n); P.Lbol.resize(n);
  P.kappa.resize(B * n); P.L.resize(B * n);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t.perm[s];
    P.rho[s] = rho[i];
    P.h[s] = std::cbrt(t.m[s] / P.rho[s]);
    double lb = 0.0;
    for (int b = 0; b < B; ++b) {
      P.kappa[b * n + s] = kappa[(int64_t)b * n + i];
      P.L[b * n + s] = lum[(int64_t)b * n + i];
      lb += P.L[b * n + s];
    }
    P.Lbol[s] = lb;
  }
}

template <>
void particle_props<Dual>(const Tree& t, const double* rho, const double* kappa, const double* lum,
                          const double* trho, const double* tkappa, const double* tlum, PartT<Dual>& P) {
  const int64_t n = t.n;
  const int B = t.B;
  P.rho.resize(n); P.h.resize(n); P.Lbol.resize(n);
  P.kappa.resize(B * n); P.L.resize(B * n);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t.perm[s];
    P.rho[s] = Dual(rho[i], trho ? trho[i] : 0.0);
    P.h[s] = cbrt(Dual(t.m[s]) / P.rho[s]);
    Dual lb(0.0);
    for (int b = 0; b < B; ++b) {
      int64_t gi = (int64_t)b * n + i;
      P.kappa[b * n + s] = Dual(kappa[gi], tkappa ? tkappa[gi] : 0.0);
      P.L[b * n + s] = Dual(lum[gi], tlum ? tlum[gi] : 0.0);
      lb += P.L[b * n + s];
    }
    P.Lbol[s] = lb;
  }
}

// ------------------------------------------------------------ geometry ----
inline double dist2_box(const double lo[3], const double hi[3], const double c[3]) {
  double dd[3];
  for (int a = 0; a < 3; ++a)
    dd[a] = (c[a] < lo[a]) ? lo[a] - c[a] : (c[a] > hi[a] ? c[a] - hi[a] : 0.0);
  return dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
}
inline double far2_box(const double lo[3], const double hi[3], const double c[3]) {
  double e[3];
  for (int a = 0; a < 3; ++a) {
    double u = lo[a] - c[a], w = hi[a] - c[a];
    e[a] = std::max(u * u, w * w);
  }
  return e[0] + e[1] + e[2];
}
inline double dist2_pt(const double* a, const double* b) {
  double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}

// Opening criterion, Section 2.5.2: open when the cell reaches into the p-p
// sphere (d < r_pp) or when B/d > theta, with d the distance from the bucket
// centre c to the nearest point of the cell and B the largest distance from
// the luminosity centre cn to the cell boundary (a corner).  Compared as
// squares: B^2 > theta^2 d^2 (equality accepts the cell).
inline bool open_cell(const double lo[3], const double hi[3], const double cn[3],
                      const double c[3], double r2, double theta2) {
  double d2 = dist2_box(lo, hi, c);
  double e[3];
  for (int a = 0; a < 3; ++a) {
    double u = cn[a] - lo[a], w = hi[a] - cn[a];
    e[a] = std::max(u * u, w * w);
  }
  double B2 = e[0] + e[1] + e[2];
  return (d2 < r2) || (B2 > theta2 * d2);
}

// Ray c + t n against an axis-aligned box: entry/exit distances (slabs).
inline bool slab(const double lo[3], const double hi[3], const double c[3], const double n[3],
                 const double inv[3], double& tin, double& tout) {
  tin = -std::numeric_limits<double>::infinity();
  tout = std::numeric_limits<double>::infinity();
  for (int a = 0; a < 3; ++a) {
    if (n[a] != 0.0) {
      double t1 = (lo[a] - c[a]) * inv[a];
      double t2 = (hi[a] - c[a]) * inv[a];
      tin = std::max(tin, std::min(t1, t2));
      tout = std::min(tout, std::max(t1, t2));
    } else if (c[a] < lo[a] || c[a] > hi[a]) {
      return false;
    }
  }
  return tin < tout;
}

// -------------------------------------------------- per-bucket computation --
template <class T> struct AbsE { T t0; double t1; int64_t node; };
template <class T> struct SrcE {
  T s;                 // projected distance on the ray
  T p[3];              // position
  std::vector<T> L;    // luminosity per band
  T d;                 // complex source model: length of the source's own ray
  std::vector<T> tin;  // complex source model: optical depth along it, per band
};

struct BucketInfo { double rpp; int64_t nnear, cells, nabs, nsrc; };

void gather_near(const Tree& t, int64_t nd, const double c[3], double r2, std::vector<int64_t>& out) {
  const NodeG& g = t.node[nd];
  // Conservative pruning (a particle can sit an ulp outside its box because
  // of rounding in the quantisation); membership is the exact test below.
  if (dist2_box(g.lo, g.hi, c) > r2 * (1.0 + 1e-9)) return;
  if (g.leaf) {
    for (int64_t s = g.first; s < g.first + g.count; ++s)
      if (dist2_pt(&t.x[3 * s], c) < r2) out.push_back(s);
    return;
  }
  gather_near(t, g.c0, c, r2, out);
  gather_near(t, g.c1, c, r2, out);
}

template <class T> struct Walker {
  const Tree& t;
  const PartT<T>& P;
  const Mom<T>& mo;
  double c[3];
  T r;
  double r2, theta2;
  std::vector<double> dir;  // [nray][3] ray directions of this bucket
  std::vector<double> inv;  // [nray][3]
  std::vector<std::vector<AbsE<T>>> abs;
  std::vector<std::vector<SrcE<T>>> src;
  int64_t cells = 0;

  Walker(const Tree& tt, const PartT<T>& PP, const Mom<T>& m) : t(tt), P(PP), mo(m) {}

  void add_absorber(int64_t nd) {
    const NodeG& g = t.node[nd];
    const double rv = val(r);
    for (int k = 0; k < t.nray; ++k) {
      double tin, tout;
      if (!slab(g.lo, g.hi, c, &dir[3 * k], &inv[3 * k], tin, tout)) continue;
      if (!(tout > std::max(tin, rv))) continue;  // nothing beyond the p-p sphere
      AbsE<T> e;
      e.t0 = (tin < rv) ? r : T(tin);
      e.t1 = tout;
      e.node = nd;
      abs[k].push_back(e);
    }
  }

  // A source at p is assigned to the ray whose pixel contains the direction
  // from the bucket centre, at the distance projected on that ray.  With
  // the complex source model a merged cell source (node >= 0) carries the
  // length and optical depth of its own ray toward the receiver (emission
  // direction -n_k, the antipodal pixel).
  void add_source(const T p[3], const T* L, int64_t node = -1) {
    T v[3];
    for (int a = 0; a < 3; ++a) v[a] = p[a] - c[a];
    int k = 0;
    T s = T(0.0);
    if (!(val(v[0]) == 0.0 && val(v[1]) == 0.0 && val(v[2]) == 0.0)) {
      k = t.hp.pixel(val(v[0]), val(v[1]), val(v[2]));
      const double* n = &dir[3 * k];
      s = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    }
    SrcE<T> e;
    e.s = s;
    for (int a = 0; a < 3; ++a) e.p[a] = p[a];
    e.L.assign(L, L + t.B);
    e.d = T(0.0);
    e.tin.assign(t.B, T(0.0));
    if (node >= 0 && (t.p.flags & F_CPLX)) {
      const int ka = t.antipode[k];
      e.d = mo.cd[node * t.nray + ka];
      for (int b = 0; b < t.B; ++b) e.tin[b] = mo.ca[(node * t.nray + ka) * t.B + b] * e.d;
    }
    src[k].push_back(e);
  }

  // Tree walk, Sections 2.5-2.5.2: open a cell if it reaches into the p-p
  // sphere or if B/d > theta (d from the bucket centre to the nearest point
  // of the cell, B from the luminosity centre to the farthest corner).  Cells
  // wholly inside the p-p sphere are left to the particle-particle part.  An
  // opened bucket contributes its volume-averaged absorption and resolves its
  // sources into particles (those outside the p-p sphere).
  void walk(int64_t nd) {
    const NodeG& g = t.node[nd];
    if (far2_box(g.lo, g.hi, c) < r2) return;
    double cn[3] = {val(mo.cen[nd * 3 + 0]), val(mo.cen[nd * 3 + 1]), val(mo.cen[nd * 3 + 2])};
    bool opened = open_cell(g.lo, g.hi, cn, c, r2, theta2);
    if (opened && !g.leaf) {
      walk(g.c0);
      walk(g.c1);
      return;
    }
    ++cells;
    if (mo.kmass[nd] > 0.0) add_absorber(nd);
    if (opened) {
      for (int64_t s = g.first; s < g.first + g.count; ++s) {
        if (!(val(P.Lbol[s]) > 0.0)) continue;
        if (dist2_pt(&t.x[3 * s], c) < r2) continue;
        T p[3] = {T(t.x[3 * s]), T(t.x[3 * s + 1]), T(t.x[3 * s + 2])};
        std::vector<T> L(t.B);
        for (int b = 0; b < t.B; ++b) L[b] = P.L[b * t.n + s];
        add_source(p, L.data());
      }
    } else if (val(mo.Lbol[nd]) > 0.0) {
      add_source(&mo.cen[nd * 3], &mo.Lb[nd * t.B], nd);
    }
  }

  // Optical depth accumulated along ray k up to distance s (order-free: the
  // priority queue of the paper only orders the same sum).
  T tau_to(int k, const T& s, int b) const {
    T tau = T(0.0);
    const int D = t.ndir, B = t.B;
    for (const AbsE<T>& e : abs[k]) {
      T end = (val(s) < e.t1) ? s : T(e.t1);
      if (!(val(end) > val(e.t0))) continue;
      tau += mo.alpha[(e.node * D + t.dir_of_ray[k]) * B + b] * (end - e.t0);
    }
    return tau;
  }
};

template <class T>
void eval_bucket(const Tree& t, const PartT<T>& P, const Mom<T>& mo, int64_t leaf,
                 const uint8_t* act_sorted, const double* bg, T* J, int64_t* cnt,
                 BucketInfo* info) {
  const Params& p = t.p;
  const NodeG& g = t.node[leaf];
  const int B = t.B, K = t.nray;
  Walker<T> W(t, P, mo);
  for (int a = 0; a < 3; ++a) W.c[a] = 0.5 * (g.lo[a] + g.hi[a]);  // bucket centre
  W.theta2 = p.theta * p.theta;
  // Ray directions: the HEALPix centres.  Directed rays (Sections 3.4.1, 4):
  // the ray whose pixel holds the direction from the bucket centre to the
  // target point is aimed exactly at it (its transmission averages stay
  // those of its HEALPix direction).
  W.dir = t.hp.v;
  if (p.flags & F_DIRECTED) {
    double v[3] = {p.target[0] - W.c[0], p.target[1] - W.c[1], p.target[2] - W.c[2]};
    if (!(v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0)) {
      double d = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      int kd = t.hp.pixel(v[0], v[1], v[2]);
      for (int a = 0; a < 3; ++a) W.dir[3 * kd + a] = v[a] / d;
    }
  }
  W.inv.resize(3 * K);
  for (int k = 0; k < K; ++k)
    for (int a = 0; a < 3; ++a) {
      double na = W.dir[3 * k + a];
      W.inv[3 * k + a] = (na != 0.0) ? 1.0 / na : 0.0;
    }
  // p-p radius (Section 2.4): a sphere about the bucket centre reaching past
  // every bucket member by its size h, grown until no particle inside it is
  // wider than the beam there (width 2 tan(theta_b) r with the beam's
  // equal-area half angle cos(theta_b) = 1 - 2/N_ray).
  std::vector<int64_t> nearv;
  T r = T(0.0);
  if (p.flags & F_NEAR) {
    const double w = 2.0 * std::tan(std::acos(1.0 - 2.0 / K));
    r = T(p.rpp_min);
    for (int64_t s = g.first; s < g.first + g.count; ++s)
      r = vmax(r, std::sqrt(dist2_pt(&t.x[3 * s], W.c)) + P.h[s]);
    for (;;) {
      double r2 = val(r) * val(r);
      nearv.clear();
      gather_near(t, 0, W.c, r2, nearv);
      T rn = r;
      for (int64_t j : nearv) rn = vmax(rn, P.h[j] / w);
      if (!(val(rn) > val(r))) break;
      r = rn;
    }
  }
  W.r = r;
  W.r2 = val(r) * val(r);
  W.abs.assign(K, {});
  W.src.assign(K, {});
  W.walk(0);

  // Optical depth to each far source (per bucket, band) and to the root-cube
  // exit of each ray (background).
  std::vector<std::vector<std::vector<T>>> tau_src(K);
  int64_t nabs = 0, nsrc = 0;
  for (int k = 0; k < K; ++k) {
    nabs += (int64_t)W.abs[k].size();
    nsrc += (int64_t)W.src[k].size();
    tau_src[k].resize(W.src[k].size());
    for (size_t e = 0; e < W.src[k].size(); ++e) {
      tau_src[k][e].resize(B);
      // the cell absorption up to the source (complex source model: up to
      // the edge of the source's cell, the projected end of its own ray)
      const SrcE<T>& S = W.src[k][e];
      for (int b = 0; b < B; ++b) tau_src[k][e][b] = W.tau_to(k, S.s - S.d, b);
    }
  }
  std::vector<T> tau_bg;
  if ((p.flags & F_BG) && bg) {
    tau_bg.resize(K * B);
    double rlo[3], rhi[3];
    for (int a = 0; a < 3; ++a) { rlo[a] = t.lo[a]; rhi[a] = t.lo[a] + t.L; }
    for (int k = 0; k < K; ++k) {
      double tin, tout;
      slab(rlo, rhi, W.c, &W.dir[3 * k], &W.inv[3 * k], tin, tout);
      for (int b = 0; b < B; ++b) tau_bg[k * B + b] = W.tau_to(k, T(tout), b);
    }
  }

  int64_t nact = 0, nhits = 0;
  std::vector<T> tpp(K * B);
  for (int64_t i = g.first; i < g.first + g.count; ++i) {
    if (!act_sorted[i]) continue;
    ++nact;
    const double* xi = &t.x[3 * i];
    const T hi = P.h[i];
    // p-p optical depth along each ray from the receiver (Section 2.4): every
    // p-p particle ahead of the receiver on the ray and within its own size
    // of the ray line adds kappa * Sigma(b); the receiver itself is excluded.
    for (int k = 0; k < K; ++k) {
      const double* n = &W.dir[3 * k];
      for (int b = 0; b < B; ++b) tpp[k * B + b] = T(0.0);
      for (int64_t l : nearv) {
        if (l == i) continue;
        const double* xl = &t.x[3 * l];
        double d[3] = {xl[0] - xi[0], xl[1] - xi[1], xl[2] - xi[2]};
        double proj = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
        if (!(proj > 0.0)) continue;
        double cx = d[1] * n[2] - d[2] * n[1];
        double cy = d[2] * n[0] - d[0] * n[2];
        double cz = d[0] * n[1] - d[1] * n[0];
        double bb = std::sqrt(cx * cx + cy * cy + cz * cz);
        if (!(bb < val(P.h[l]))) continue;
        T sig = column_sigma(bb, t.m[l], P.h[l]);
        for (int b = 0; b < B; ++b) tpp[k * B + b] += P.kappa[b * t.n + l] * sig;
      }
    }
    std::vector<T> Jb(B, T(0.0));
    // Far sources (Section 2.5.1): attenuated by the receiver's p-p column on
    // the ray and by the cell optical depth up to the source's projected
    // distance, scaled by true over projected distance.
    for (int k = 0; k < K; ++k) {
      for (size_t e = 0; e < W.src[k].size(); ++e) {
        const SrcE<T>& S = W.src[k][e];
        T dx = S.p[0] - xi[0], dy = S.p[1] - xi[1], dz = S.p[2] - xi[2];
        T rr = sqrt(dx * dx + dy * dy + dz * dz);
        T Kv = kernel_K(rr, hi);
        for (int b = 0; b < B; ++b) {
          T tc = tau_src[k][e][b];
          T ex = (val(tc) > 0.0) ? tc * rr / S.s : T(0.0);
          Jb[b] += S.L[b] * Kv * exp(-tpp[k * B + b] - ex - S.tin[b]);
        }
      }
    }
    // Near sources (Section 2.4), including the receiver itself at r = 0:
    // absorbed by p-p particles closer to the source than the receiver is,
    // within their size of the receiver-source segment.
    for (int64_t j : nearv) {
      if (!(val(P.Lbol[j]) > 0.0)) continue;
      const double* xj = &t.x[3 * j];
      double rij2 = dist2_pt(xi, xj);
      double rij = std::sqrt(rij2);
      T Kv = kernel_K(T(rij), hi);
      std::vector<T> tau(B, T(0.0));
      double e[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
      for (int64_t l : nearv) {
        if (l == i || l == j) continue;
        const double* xl = &t.x[3 * l];
        if (!(dist2_pt(xl, xj) < rij2)) continue;
        double w[3] = {xl[0] - xi[0], xl[1] - xi[1], xl[2] - xi[2]};
        double u = (w[0] * e[0] + w[1] * e[1] + w[2] * e[2]) / rij2;
        u = std::min(1.0, std::max(0.0, u));
        double f[3] = {w[0] - u * e[0], w[1] - u * e[1], w[2] - u * e[2]};
        double bb = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (!(bb < val(P.h[l]))) continue;
        ++nhits;
        T sig = column_sigma(bb, t.m[l], P.h[l]);
        for (int b = 0; b < B; ++b) tau[b] += P.kappa[b * t.n + l] * sig;
      }
      for (int b = 0; b < B; ++b) Jb[b] += P.L[b * t.n + j] * Kv * exp(-tau[b]);
    }
    // Isotropic background entering at the root-cube boundary: each ray
    // carries 4 pi / N_ray of it, attenuated along the whole ray.
    if ((p.flags & F_BG) && bg) {
      for (int k = 0; k < K; ++k)
        for (int b = 0; b < B; ++b)
          Jb[b] += (4.0 * kPi / K) * bg[b] *
                   exp(-tpp[k * B + b] - tau_bg[k * B + b]);
    }
    // Element-averaged intensity of an optically thick element (Section 2.1).
    for (int b = 0; b < B; ++b) {
      if (p.flags & F_THICK) Jb[b] = Jb[b] * thick_C(P.kappa[b * t.n + i] * P.rho[i] * hi);
      J[(int64_t)b * t.n + t.perm[i]] = Jb[b];
    }
  }
  cnt[C_BUCKETS] += 1;
  cnt[C_CELLS] += W.cells;
  cnt[C_ABS] += nabs;
  cnt[C_SRC] += nsrc;
  cnt[C_SEG] += nact * ((int64_t)K + nabs + nsrc);
  cnt[C_NEAR_PAIRS] += nact * (int64_t)nearv.size();
  cnt[C_SRC_PAIRS] += nact * nsrc;
  int64_t nlum = 0;
  for (int64_t j : nearv) nlum += (val(P.Lbol[j]) > 0.0) ? 1 : 0;
  cnt[C_NS_TRIPLES] += nact * nlum * (int64_t)nearv.size();
  cnt[C_NS_HITS] += nhits;
  cnt[C_MAX_NEAR] = std::max<int64_t>(cnt[C_MAX_NEAR], (int64_t)nearv.size());
  if (info) {
    info->rpp = val(r);
    info->nnear = (int64_t)nearv.size();
    info->cells = W.cells;
    info->nabs = nabs;
    info->nsrc = nsrc;
  }
}

struct Handle {
  Tree* t;
  PartT<double> P;
  Mom<double> mo;
};

template <class T>
void run_all(const Tree& t, const PartT<T>& P, const Mom<T>& mo, const uint8_t* active,
             const double* bg, T* J, int64_t* counters, double* bucket_info, int nthreads) {
  std::vector<uint8_t> act(t.n);
  for (int64_t s = 0; s < t.n; ++s) act[s] = active ? (active[t.perm[s]] ? 1 : 0) : 1;
  std::vector<int64_t> leaves;
  for (int64_t nd = 0; nd < (int64_t)t.node.size(); ++nd) {
    const NodeG& g = t.node[nd];
    if (!g.leaf) continue;
    bool any = false;
    for (int64_t s = g.first; s < g.first + g.count; ++s) any = any || act[s];
    if (any) leaves.push_back(nd);
  }
  int64_t cnt[C_N] = {0};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    int64_t loc[C_N] = {0};
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
    for (int64_t bi = 0; bi < (int64_t)leaves.size(); ++bi) {
      BucketInfo inf;
      eval_bucket(t, P, mo, leaves[bi], act.data(), bg, J, loc, bucket_info ? &inf : nullptr);
      if (bucket_info) {
        double* o = bucket_info + 6 * bi;
        o[0] = (double)leaves[bi];
        o[1] = inf.rpp;
        o[2] = (double)inf.nnear;
        o[3] = (double)inf.cells;
        o[4] = (double)inf.nabs;
        o[5] = (double)inf.nsrc;
      }
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    {
      for (int c = 0; c < C_N; ++c)
        if (c == C_MAX_NEAR) cnt[c] = std::max(cnt[c], loc[c]);
        else cnt[c] += loc[c];
    }
  }
  cnt[C_NODES] = (int64_t)t.node.size();
  if (counters)
    for (int c = 0; c < C_N; ++c) counters[c] = cnt[c];
}

}  // namespace

// ================================================================ C ABI ====
extern "C" {

// Unit functions (for pinning tests).
double ora_kernel_K(double r, double h) { return kernel_K<double>(r, h); }
double ora_thick_C(double tau) { return thick_C<double>(tau); }
double ora_column_sigma(double b, double m, double h) {
  return b < h ? column_sigma<double>(b, m, h) : 0.0;
}
void ora_healpix_centres(int nside, double* out) {
  Healpix hp(nside);
  std::memcpy(out, hp.v.data(), sizeof(double) * 3 * hp.npix);
}
void ora_healpix_pixel(int nside, int64_t m, const double* v, int32_t* out) {
  Healpix hp(nside);
  for (int64_t i = 0; i < m; ++i) out[i] = hp.pixel(v[3 * i], v[3 * i + 1], v[3 * i + 2]);
}
// Transmission-average combine of two half boxes (sides s, split axis a).
double ora_combine(const double* s, int a, const double* n, double a1, double a2, double* geom) {
  CombineGeom g = combine_geom(s, a, n);
  if (geom) { geom[0] = g.w1; geom[1] = g.w12; geom[2] = g.d; }
  return combine_alpha<double>(g, a1, a2);
}

int ora_open_cell(const double* lo, const double* hi, const double* cn, const double* c,
                  double r, double theta) {
  return open_cell(lo, hi, cn, c, r * r, theta * theta) ? 1 : 0;
}

void* ora_build(const Params* p, int64_t n, const double* x, const double* y, const double* z,
                const double* m, const double* rho, const double* kappa, const double* lum) {
  Handle* H = new Handle();
  H->t = build_geometry(*p, n, x, y, z, m);
  particle_props<double>(*H->t, rho, kappa, lum, nullptr, nullptr, nullptr, H->P);
  compute_moments<double>(*H->t, H->P, H->mo);
  if (p->flags & F_CPLX) complex_sources<double>(*H->t, H->mo);
  return H;
}
void ora_free(void* h) {
  Handle* H = (Handle*)h;
  delete H->t;
  delete H;
}
int64_t ora_num_nodes(void* h) { return (int64_t)((Handle*)h)->t->node.size(); }
int32_t ora_num_dirs(void* h) { return ((Handle*)h)->t->ndir; }
void ora_root(void* h, double* box4) {
  Tree* t = ((Handle*)h)->t;
  box4[0] = t->lo[0]; box4[1] = t->lo[1]; box4[2] = t->lo[2]; box4[3] = t->L;
}
void ora_dirs(void* h, int32_t* dir_of_ray, int32_t* ray_of_dir) {
  Tree* t = ((Handle*)h)->t;
  for (int k = 0; k < t->nray; ++k) dir_of_ray[k] = t->dir_of_ray[k];
  for (int j = 0; j < t->ndir; ++j) ray_of_dir[j] = t->ray_of_dir[j];
}
void ora_perm(void* h, int64_t* perm, uint64_t* keys) {
  Tree* t = ((Handle*)h)->t;
  for (int64_t s = 0; s < t->n; ++s) { perm[s] = t->perm[s]; if (keys) keys[s] = t->key[s]; }
}
// Node tables in preorder.  ints: [node][7] = first, count, lown, split, c0,
// c1, next (leaf iff split < 0).  dbl: [node][6] = lo, hi.  cen: [node][3].
// Lb: [node][B]; Lbol: [node]; kmass: [node]; alpha: [node][ndir][B].
void ora_nodes(void* h, int64_t* ints, double* box, double* cen, double* Lb, double* Lbol,
               double* kmass, double* alpha) {
  Handle* H = (Handle*)h;
  Tree* t = H->t;
  const int64_t nn = (int64_t)t->node.size();
  const int B = t->B, D = t->ndir;
  for (int64_t i = 0; i < nn; ++i) {
    const NodeG& g = t->node[i];
    int64_t* o = ints + 7 * i;
    o[0] = g.first; o[1] = g.count; o[2] = g.lown; o[3] = g.split;
    o[4] = g.c0; o[5] = g.c1; o[6] = g.next;
    for (int a = 0; a < 3; ++a) { box[6 * i + a] = g.lo[a]; box[6 * i + 3 + a] = g.hi[a]; }
    for (int a = 0; a < 3; ++a) cen[3 * i + a] = H->mo.cen[3 * i + a];
    for (int b = 0; b < B; ++b) Lb[i * B + b] = H->mo.Lb[i * B + b];
    Lbol[i] = H->mo.Lbol[i];
    kmass[i] = H->mo.kmass[i];
  }
  if (alpha) std::memcpy(alpha, H->mo.alpha.data(), sizeof(double) * nn * D * B);
}
// Complex source model tables (nodes in preorder): cd [node][nray] lengths,
// ca [node][nray][B] absorption coefficients; antipode [nray].  Zeros when
// the model is off.
void ora_complex(void* h, double* cd, double* ca, int32_t* antipode) {
  Handle* H = (Handle*)h;
  Tree* t = H->t;
  const size_t nn = t->node.size(), K = (size_t)t->nray, B = (size_t)t->B;
  for (size_t i = 0; i < nn * K; ++i) cd[i] = H->mo.cd.empty() ? 0.0 : H->mo.cd[i];
  for (size_t i = 0; i < nn * K * B; ++i) ca[i] = H->mo.ca.empty() ? 0.0 : H->mo.ca[i];
  for (size_t k = 0; k < K; ++k) antipode[k] = t->antipode[k];
}

// J [B][n] in input order (rows of inactive particles untouched).
// counters[11]: buckets, cells, absorber entries, source entries, segments,
// near pairs, largest near set, nodes, receiver-source pairs, p-p source
// path tests, p-p source path hits (element within its size of the segment
// and nearer the source than the receiver).  bucket_info (optional) [nb][6]:
// leaf node, r_pp, near count, cells, absorber entries, source entries.
int64_t ora_compute_J(void* h, const uint8_t* active, const double* bg, double* J,
                      int64_t* counters, double* bucket_info, int nthreads) {
  Handle* H = (Handle*)h;
  run_all<double>(*H->t, H->P, H->mo, active, bg, J, counters, bucket_info, nthreads);
  return 0;
}
// One-shot forward-mode derivative: J and dJ = (dJ/dL) tL + (dJ/dkappa) tk +
// (dJ/drho) trho with every discrete decision frozen at the values.
int64_t ora_jvp(const Params* p, int64_t n, const double* x, const double* y, const double* z,
                const double* m, const double* rho, const double* kappa, const double* lum,
                const uint8_t* active, const double* bg, const double* tL, const double* tk,
                const double* trho, double* J, double* dJ, int64_t* counters, int nthreads) {
  Tree* t = build_geometry(*p, n, x, y, z, m);
  PartT<Dual> P;
  particle_props<Dual>(*t, rho, kappa, lum, trho, tk, tL, P);
  Mom<Dual> mo;
  compute_moments<Dual>(*t, P, mo);
  if (p->flags & F_CPLX) complex_sources<Dual>(*t, mo);
  std::vector<Dual> Jd((size_t)t->B * n);
  for (size_t i = 0; i < Jd.size(); ++i) Jd[i] = Dual(J[i], dJ[i]);
  run_all<Dual>(*t, P, mo, active, bg, Jd.data(), counters, nullptr, nthreads);
  for (size_t i = 0; i < Jd.size(); ++i) { J[i] = Jd[i].v; dJ[i] = Jd[i].d; }
  delete t;
  return 0;
}

}  // extern "C"
