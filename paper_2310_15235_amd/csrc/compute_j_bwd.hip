// Adjoint of the mean intensity path: given dE/dJ, the gradients dE/dL,
// dE/dkappa and dE/drho (Sections 2.1-2.6 of Wadsley, Baumschlager & Shen
// 2023 define the forward map; its derivative is taken with every discrete
// decision held fixed: tree, opening, pixel of a source, p-p membership,
// which element sets the p-p radius, which cells a ray crosses).
//
// The forward decisions are recomputed by the forward's own code (bucket
// setup, walk, p-p optical depths), then each stage is swept in reverse:
//   k_pp_src_bwd   p-p sources: dL_j, dh_i through K, dkappa_l and dh_l
//                  through the columns on the source paths; the p-p part of
//                  the raw J (needed by the thick-element factor);
//   k_far_bwd      far sources and background: the optical depths are
//                  recomputed, then per (receiver, source) the adjoints of the
//                  p-p optical depth per (receiver, ray), of each source's cell
//                  optical depth, luminosity and position, of h_i; a second
//                  sweep over the hits turns the source optical-depth
//                  adjoints into cell-absorption adjoints (per node, direction
//                  class and band) and the p-p radius adjoint; the
//                  thick-element factor;
//   k_pp_rays_bwd  p-p columns per (receiver, ray): dkappa_l, dh_l;
//   k_rpp_bwd      the p-p radius adjoint to the size of the element that set
//                  it (member reach |x - c| + h, or h/w while growing);
//   tree kernels   top-down through the transmission combine, the bucket
//                  absorption sum(kappa m)/sum(m/rho), luminosity sums and
//                  luminosity centres; then h = (m/rho)^(1/3) and input order.
// Per-term arithmetic is FP32 like the forward; sums of many terms and all
// gradient accumulators are FP64 (hardware FP64 atomics where several
// buckets meet).

#include <algorithm>
#include <cmath>

#include "path_device.hpp"
#include "path_host.hpp"

namespace trevr {

__device__ inline double* galpha_copy(const Grad& G) {
  return G.galpha + (int64_t)(blockIdx.x & (G.ka - 1)) * G.na;
}
__device__ inline double* gLb_copy(const Grad& G) {
  return G.gLb + (int64_t)(blockIdx.x & (G.ks - 1)) * G.ns;
}
__device__ inline double* gcen_copy(const Grad& G) {
  return G.gcen + (int64_t)(blockIdx.x & (G.ks - 1)) * G.nc;
}

__device__ inline void gadd(double* a, double v) {
  if (v != 0.0) unsafeAtomicAdd(a, v);
}

// d f/d x of the intensity kernel shape f (see fshape): below 1/2 and from 2
// on by the derivatives of the series 2 - sum 2 x^2k/(4k^2-1) and
// sum 2 x^-2k/(4k^2-1); in between 1/x - (1 + x^2) atanh(x^+-1)/x^2.
__device__ inline float fshape_d(float x) {
  if (x < 0.5f) {
    const float y = x * x;
    float s = 44.0f / 483.0f;
    s = __builtin_fmaf(s, y, 40.0f / 399.0f);
    s = __builtin_fmaf(s, y, 36.0f / 323.0f);
    s = __builtin_fmaf(s, y, 32.0f / 255.0f);
    s = __builtin_fmaf(s, y, 28.0f / 195.0f);
    s = __builtin_fmaf(s, y, 24.0f / 143.0f);
    s = __builtin_fmaf(s, y, 20.0f / 99.0f);
    s = __builtin_fmaf(s, y, 16.0f / 63.0f);
    s = __builtin_fmaf(s, y, 12.0f / 35.0f);
    s = __builtin_fmaf(s, y, 8.0f / 15.0f);
    s = __builtin_fmaf(s, y, 4.0f / 3.0f);
    return -x * s;
  }
  if (x < 1.0f) {
    const float at = 0.5f * log1pf(2.0f * x / (1.0f - x));
    return 1.0f / x - (1.0f + x * x) * at / (x * x);
  }
  if (x < 2.0f) {
    if (x == 1.0f) return 0.0f;
    const float at = 0.5f * logf((x + 1.0f) / (x - 1.0f));
    return 1.0f / x - (1.0f + x * x) * at / (x * x);
  }
  const float y = __builtin_amdgcn_rcpf(x * x);
  float s = 44.0f / 483.0f;
  s = __builtin_fmaf(s, y, 40.0f / 399.0f);
  s = __builtin_fmaf(s, y, 36.0f / 323.0f);
  s = __builtin_fmaf(s, y, 32.0f / 255.0f);
  s = __builtin_fmaf(s, y, 28.0f / 195.0f);
  s = __builtin_fmaf(s, y, 24.0f / 143.0f);
  s = __builtin_fmaf(s, y, 20.0f / 99.0f);
  s = __builtin_fmaf(s, y, 16.0f / 63.0f);
  s = __builtin_fmaf(s, y, 12.0f / 35.0f);
  s = __builtin_fmaf(s, y, 8.0f / 15.0f);
  s = __builtin_fmaf(s, y, 4.0f / 3.0f);
  return -s * y * __builtin_amdgcn_rcpf(x);
}

// Thick-element factor C(tau) = (1 - e^-tau)/tau (Section 2.1) and C'(tau).
__device__ inline double thick_C(double tau) { return tau == 0.0 ? 1.0 : -expm1(-tau) / tau; }
__device__ inline double thick_dC(double tau) {
  if (tau < 1e-3) return -0.5 + tau * (1.0 / 3.0 + tau * (-0.125 + tau * (1.0 / 30.0)));
  return (exp(-tau) - thick_C(tau)) / tau;
}

// Per receiver of a chunk: w_ib = dE/dJ_ib C_ib (the adjoint of the raw J)
// and 1/h_i.  Threads t < nrecv * NB.
template <int NB>
__device__ inline void load_receiver_adjoints(const DevTree& T, const double* gJ,
                                              const RecvInfo* recv, int nrecv, float (*gw)[NB],
                                              float* rinvh) {
  const int t = threadIdx.x;
  const int64_t n = T.n;
  if (t < nrecv * NB) {
    const int i = t / NB, b = t % NB;
    const uint32_t sl = recv[i].slot;
    double C = 1.0;
    if (T.flags & TREVR_THICK_CORR)
      C = thick_C((double)T.kappa[(int64_t)b * n + sl] * (double)T.rho[sl] * recv[i].h);
    gw[i][b] = (float)(gJ[(int64_t)b * n + T.perm[sl]] * C);
  }
  if (t < nrecv) rinvh[t] = (float)(1.0 / recv[t].h);
  __syncthreads();
}

// ------------------------------------------------------ p-p sources
// Adjoint of k_pp_src, with the pair optical depths tau_ijb the forward
// left in ptau.  Per pass of up to kNT (receiver i, luminous p-p element j)
// pairs: each thread takes a pair, term_b = L_jb K(r_ij, h_i) e^{-tau_ijb};
// dL_jb += w_ib K e_b, dh_i += w_ib L_jb e_b dK/dh, and the column adjoint
// gt_b = -w_ib term_b goes to LDS with the pair.  Then element-major: each
// thread takes a p-p element l, sweeps the staged pairs (groups of 16
// culled by their segments' bounding box), decides "l absorbs on i-j" with
// the forward's FP64 operation sequence and sums dkappa_lb += gt_b Sigma_l,
// dh_l += gt_b kappa_lb dSigma_l/dh_l in registers.  The p-p part of the
// raw J goes to jraw per receiver.
template <int NB> struct PairTile {
  float xj[kNT][3];   // FP32 as stored, widened where read
  double rij2[kNT], inv2[kNT];
  float gt[kNT][NB];
  uint32_t j[kNT];
  // the source of each pair relative to the bucket centre and its run's
  // test values (RunTab): every receiver's segment to the source lies within
  // the round cone of the receivers' reach around the centre's segment
  float jr[kNT][3], jinv[kNT], jlim[kNT], k2[kNT], m2[kNT];
};


template <int NB>
__global__ void __launch_bounds__(kNT, 4) k_pp_src_bwd(const DevTree* __restrict__ TT, Items I,
                                                   const uint32_t* blist, const uint32_t* bscene,
                                                   const uint32_t* noff, const uint32_t* nlumc,
                                                   const uint32_t* nidx, const uint32_t* joff,
                                                   const uint32_t* poff, const float* ptau,
                                                   const uint8_t* active, const double* gJall,
                                                   Grad Gall, double* jraw, JobLog JL) {
  const int t = threadIdx.x;
  __shared__ PairTile<NB> PT;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, s_item;
  __shared__ float gw[kRMax][NB], rinvh[kRMax];
  __shared__ double red[kNT][NB];
  __shared__ double redh[kNT];
  __shared__ uint16_t jobq[kNT / 64][2][kJobQ];   // per wavefront: (element lane, source run)
  __shared__ float eacc[kNT / 64][64][NB + 1];     // per wavefront: element sums
  __shared__ float egrp[kNT / 64][4][5];   // per wavefront: element spheres of its quarters
  const int lane = t & 63, wv = t >> 6;
  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  const double* gJ = gJall + T.joff;
  const Grad G = Gall.at(T);
  double* jrawb = jraw + joff[bucket];
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0, nl = nlumc[bucket];
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int64_t n = T.n;
  uint32_t member = lk.x;
  uint32_t nact = 0;
  // the forward's job log of this bucket, where it covers it: the element-
  // major sweep then reads its jobs instead of culling again
  const bool logged = JL.log && JL.tab[4 * bucket].x != kLogNone;
  LogPos lp{0u, 0u};
  if (logged) {
    const uint2 s = JL.tab[4 * bucket + wv];
    lp.blk = (uint32_t)__builtin_amdgcn_readfirstlane((int)(s.x < JL.blocks ? s.x : 0u));
    lp.pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)min(s.y, kLogData));
  }
  for (;;) {
    const int nrecv = load_receivers(T, act, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    load_receiver_adjoints<NB>(T, gJ, recv, nrecv, gw, rinvh);
    const float* pt = ptau + (int64_t)poff[bucket] + (int64_t)nact * nl * NB;
    const int stride = (kNT / nrecv) * nrecv;       // thread t keeps receiver t % nrecv
    const int i = t % nrecv;
    const RecvInfo& ri = recv[i];
    float reach = 0.0f;   // largest receiver distance from the centre
    for (int k = 0; k < nrecv; ++k)
      reach = fmaxf(reach, sqrtf(recv[k].rel[0] * recv[k].rel[0] + recv[k].rel[1] * recv[k].rel[1] +
                                 recv[k].rel[2] * recv[k].rel[2]));
    // each thread's sums over its pairs (its own LDS slots, registers stay
    // free for the sweep)
#pragma unroll
    for (int b = 0; b < NB; ++b) red[t][b] = 0.0;
    redh[t] = 0.0;
    const uint32_t P = (uint32_t)nrecv * nl;
    for (uint32_t pb = 0; pb < P; pb += (uint32_t)stride) {
      // ---- pairs: terms and column adjoints
      const uint32_t p = pb + (uint32_t)t;
      const bool ok = t < stride && p < P;
      const uint32_t j = ok ? near[p / nrecv] : near[0];
      const double xj0 = (double)T.x[j], xj1 = (double)T.y[j], xj2 = (double)T.z[j];
      const double e0 = xj0 - ri.x[0], e1 = xj1 - ri.x[1], e2 = xj2 - ri.x[2];
      const double rij2 = e0 * e0 + e1 * e1 + e2 * e2;
      bool valid = false;
      float gt[NB];
      double gl[NB];   // luminosity adjoint of source j from this pair
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        gt[b] = 0.0f;
        gl[b] = 0.0;
      }
      if (ok) {
        const float x = (float)sqrt(rij2) * ri.inv_rh;
        const float f = fshape(x);
        const float Kv = f * ri.kfac;
        const float dKdh = -(2.0f * f + x * fshape_d(x)) * ri.kfac * rinvh[i];
        double ghi = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double E = exp(-(double)pt[(int64_t)p * NB + b]);
          const double Lj = (double)T.lum[(int64_t)b * n + j];
          const double term = Lj * (double)Kv * E;
          red[t][b] += term;
          const double w = (double)gw[i][b];
          gl[b] = w * (double)Kv * E;
          ghi += w * Lj * E * (double)dKdh;
          gt[b] = (float)(-w * term);
          valid = valid || gt[b] != 0.0f;
        }
        redh[t] += ghi;
      }
      {
        // the nrecv pairs of one source sit on consecutive lanes: the first
        // lane of each run (or of its part in this wavefront) adds the run's
        // sum, one atomic per source and band instead of one per pair
        const uint32_t k0 = p % (uint32_t)nrecv;
        const bool head = k0 == 0u || lane == 0;
        double g0[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) g0[b] = gl[b];
        for (int k = 1; k < nrecv; ++k) {
          const bool same = k0 + (uint32_t)k < (uint32_t)nrecv && lane + k < 64;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const double v = __shfl_down(g0[b], (unsigned)k);
            if (same) gl[b] += v;
          }
        }
        if (ok && head) {
#pragma unroll
          for (int b = 0; b < NB; ++b) gadd(&G.gL[(int64_t)b * n + j], gl[b]);
        }
      }
      if (ok) {
        valid = valid && rij2 > 0.0;
      }
      PT.xj[t][0] = (float)xj0;   // exact: the positions are FP32
      PT.xj[t][1] = (float)xj1;
      PT.xj[t][2] = (float)xj2;
      PT.rij2[t] = valid ? rij2 : -1.0;   // no adjoint or no path: fails the exact test
      PT.inv2[t] = rij2 > 0.0 ? 1.0 / rij2 : 0.0;
      {
        const float js[3] = {(float)(xj0 - c[0]), (float)(xj1 - c[1]), (float)(xj2 - c[2])};
        run_tab_entry(js, reach, PT.jr, PT.jinv, PT.jlim, PT.k2, PT.m2, t);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) PT.gt[t][b] = gt[b];
      PT.j[t] = j;
      __syncthreads();
      if (__syncthreads_or(valid)) {
        const int qend = (int)min((uint32_t)stride, P - pb);   // pairs of this pass
        const RunTab RT{PT.jr, PT.jinv, PT.jlim, PT.k2, PT.m2};
        const float Rm = reach * (1.0f + 1e-5f);
        uint16_t* QA = jobq[wv][0];   // per-element test passes
        uint16_t* Q = jobq[wv][1];    // round-cone passes: exact tests
        float (*A)[NB + 1] = eacc[wv];
        // ---- p-p elements against the staged pairs.  Each lane owns an
        // element; per source run it tests the element against the
        // cylinder of the receivers' reach around the centre's segment to
        // the source and the element no farther from the source than the
        // farthest receiver; passing jobs are filtered by the round cone
        // (the reach at the centre, none at the source).
        // Passing (element, source run) jobs are queued per wavefront and
        // run 64 at a time, so the exact FP64 tests keep every lane busy.
        // logged: the pass's records, one per chunk with jobs of this
        // wavefront, in chunk order (rc: the next one's chunk, rcnt: its jobs)
        uint32_t rleft = 0, rc = kLogNone, rcnt = 0, cnext = 0;
        auto next_record = [&]() {
          rc = kLogNone;
          if (rleft == 0u) return;
          --rleft;
          const uint32_t e2 = log_get_record(JL, lp, (uint32_t)lane);
          rc = cnext + (uint32_t)__builtin_amdgcn_readlane((int)e2, 0);
          rcnt = (uint32_t)__builtin_amdgcn_readlane((int)e2, 1);
          cnext = rc + 1u;
        };
        if (logged) {
          rleft = (uint32_t)__builtin_amdgcn_readfirstlane((int)log_get(JL, lp, 1u, 0u));
          next_record();
        }
        for (uint32_t c0 = 0; c0 < nnear; c0 += kNT) {
          // logged: only the chunks with jobs of this wavefront
          uint32_t lcnt = 0;
          if (logged) {
            if (c0 / (uint32_t)kNT != rc) continue;
            lcnt = rcnt;
          }
          const uint32_t u = c0 + (uint32_t)t;
          const bool has = u < nnear;
          const uint32_t l = has ? near[u] : near[0];
          // positions stay FP32 (as stored) until a job widens them
          const float ux = T.x[l], uy = T.y[l], uz = T.z[l];
          const double hl = T.h[l];
          const double h2 = hl * hl;
          // column density scale 3m/(pi h^2) and 1/h in FP32 (they set the
          // values added, not the decisions)
          const float iv = __builtin_amdgcn_rcpf((float)hl);
          const float sig = (float)(3.0 / kPi) * T.m[l] * iv * iv;
          float kap[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) kap[b] = T.kappa[(int64_t)b * n + l];
          const float pr[3] = {(float)((double)ux - c[0]), (float)((double)uy - c[1]),
                               (float)((double)uz - c[2])};
          // no element: a NaN size, which fails every element test
          const float hrad = has ? (float)hl * (1.0f + 1e-5f) +
                                       1e-5f * (fabsf(pr[0]) + fabsf(pr[1]) + fabsf(pr[2]))
                                 : __int_as_float(0x7fc00000);
#pragma unroll
          for (int b = 0; b <= NB; ++b) A[lane][b] = 0.0f;
          uint32_t head = 0, tail = 0, ha = 0, ta = 0;   // wave-uniform queue cursors

          // one batch of up to 64 jobs, one per lane (where mine): a job is
          // (element, source run); its lane runs the exact test of the
          // element on each of the run's nrecv pairs (pair q0 + k has
          // receiver k), the element and source read once, sums the
          // element's adjoints over the run and adds them to its LDS sums
          auto exact_jobs = [&](bool mine, uint32_t job) {
            const int L = mine ? (int)((job >> 8) & 63u) : lane;
            const int q0 = (int)(job & 0xFFu);
            const double vx = (double)__shfl(ux, L), vy = (double)__shfl(uy, L),
                         vz = (double)__shfl(uz, L);
            const double vh2 = __shfl(h2, L);
            const float vsig = __shfl(sig, L), viv = __shfl(iv, L);
            const uint32_t vl = (uint32_t)__shfl((int)l, L);
            float vkap[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) vkap[b] = __shfl(kap[b], L);
            if (mine) {
              const double qx0 = (double)PT.xj[q0][0], qx1 = (double)PT.xj[q0][1],
                           qx2 = (double)PT.xj[q0][2];
              const uint32_t qj = PT.j[q0];
              const double f0 = vx - qx0, f1 = vy - qx1, f2 = vz - qx2;
              const double ff = f0 * f0 + f1 * f1 + f2 * f2;
              float ga[NB], gh = 0.0f;
              bool any = false;
#pragma unroll
              for (int b = 0; b < NB; ++b) ga[b] = 0.0f;
              // two receivers per step, every condition evaluated: their LDS
              // reads issue together instead of one wait per condition
              // (222 -> 198 ms on the batched workload)
#pragma unroll 2
              for (int k = 0; k < nrecv; ++k) {
                const int q = q0 + k;
                const RecvInfo& rq = recv[k];
                const double xi0 = rq.x[0], xi1 = rq.x[1], xi2 = rq.x[2];
                const double e0q = qx0 - xi0, e1q = qx1 - xi1, e2q = qx2 - xi2;
                const double w0 = vx - xi0, w1 = vy - xi1, w2 = vz - xi2;
                double uu = (w0 * e0q + w1 * e1q + w2 * e2q) * PT.inv2[q];
                uu = fmin(1.0, fmax(0.0, uu));
                const double g0 = w0 - uu * e0q, g1 = w1 - uu * e1q, g2 = w2 - uu * e2q;
                const double b2 = g0 * g0 + g1 * g1 + g2 * g2;
                if ((ff < PT.rij2[q]) & (b2 < vh2) & (vl != rq.slot) &
                    (vl != qj)) {
                  const float bb = __builtin_amdgcn_sqrtf((float)b2);
                  const float sg = vsig * (1.0f - bb * viv);
                  const float dsg = vsig * viv * (3.0f * bb * viv - 2.0f);
                  float gqk = 0.0f;
#pragma unroll
                  for (int b = 0; b < NB; ++b) {
                    ga[b] += PT.gt[q][b] * sg;
                    gqk += PT.gt[q][b] * vkap[b];
                  }
                  gh += gqk * dsg;
                  any = true;
                }
              }
              if (any) {
#pragma unroll
                for (int b = 0; b < NB; ++b) atomicAdd(&A[L][b], ga[b]);
                atomicAdd(&A[L][NB], gh);
              }
            }
          };
          // the queued jobs head + lane
          auto run_jobs = [&](uint32_t cnt) {
            exact_jobs((uint32_t)lane < cnt, Q[(head + (uint32_t)lane) & (kJobQ - 1)]);
          };
          // the round-cone filter over up to 64 jobs of the first queue (job
          // ha + lane on this lane); the survivors go to the exact tests
          auto filter_jobs = [&](uint32_t cnt) {
            const bool mine = (uint32_t)lane < cnt;
            const uint16_t job = QA[(ha + (uint32_t)lane) & (kJobQ - 1)];
            const int L = mine ? (int)(job >> 8) : lane;
            const float vp[3] = {__shfl(pr[0], L), __shfl(pr[1], L), __shfl(pr[2], L)};
            const float vh = __shfl(hrad, L);
            const bool keep = mine && elem_run_cone(vp, vh, RT, Rm, (int)(job & 0xFFu));
            const uint64_t m = ballot64(keep);
            if (keep) Q[(tail + (uint32_t)mbcnt(m)) & (kJobQ - 1)] = job;
            tail += (uint32_t)__popcll(m);
            wave_lds_sync();
            while (tail - head >= 64u) {
              run_jobs(64u);
              head += 64u;
            }
          };
          if (logged) {
            // the forward's jobs of this chunk, 64 at a time
            for (uint32_t d = 0; d < lcnt; d += 64u) {
              const uint32_t cnt = min(64u, lcnt - d);
              const uint32_t job = log_get(JL, lp, cnt, (uint32_t)lane);
              exact_jobs((uint32_t)lane < cnt && (int)(job & 0xFFu) + nrecv <= qend, job);
            }
          } else {
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
                const int eL =
                    pq >= 0 ? (pq >> 4) * kElemGroup + (lane & (kElemGroup - 1)) : lane;
                const int q0 = pq >= 0 ? (k0 + (pq & (kElemGroup - 1))) * nrecv : 0;
                const float vp[3] = {__shfl(pr[0], eL), __shfl(pr[1], eL), __shfl(pr[2], eL)};
                const float vh = __shfl(hrad, eL);
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
            if (tail > head) run_jobs(tail - head);
          }
          wave_lds_sync();
          if (has) {
#pragma unroll
            for (int b = 0; b < NB; ++b) gadd(&G.gk[(int64_t)b * n + l], (double)A[lane][b]);
            gadd(&G.gh[l], (double)A[lane][NB]);
          }
          wave_lds_sync();
          if (logged) next_record();
        }
        // records of chunks past the set (none in a log the forward wrote)
        while (logged && rc != kLogNone) {
          log_skip(JL, lp, rcnt);
          next_record();
        }
      } else if (logged) {
        // no pair of this pass has an adjoint: step over its records and jobs
        uint32_t rl = (uint32_t)__builtin_amdgcn_readfirstlane((int)log_get(JL, lp, 1u, 0u));
        for (; rl > 0u; --rl) {
          const uint32_t e2 = log_get_record(JL, lp, (uint32_t)lane);
          log_skip(JL, lp, (uint32_t)__builtin_amdgcn_readlane((int)e2, 1));
        }
      }
      __syncthreads();
    }
    // receiver-wise sums in thread order
    __syncthreads();
    if (t < nrecv * NB) {
      const int ii = t / NB, b = t % NB;
      double v = 0.0;
      for (int u = ii; u < stride; u += nrecv) v += red[u][b];
      jrawb[(int64_t)(nact + ii) * NB + b] = v;
    }
    if (t < nrecv) {
      double v = 0.0;
      for (int u = t; u < stride; u += nrecv) v += redh[u];
      gadd(&G.gh[recv[t].slot], v);
    }
    nact += (uint32_t)nrecv;
    __syncthreads();
  }
  }
}

// ------------------------------------------------------ p-p columns
// Adjoint of k_pp_rays: tau_ikb = sum_l kappa_lb Sigma_l(b_ilk) with the
// adjoint g_ikb of the far-field kernel: dkappa_lb += g Sigma, dh_l +=
// g kappa_lb dSigma/dh.  Element-major: threads take (p-p element l,
// receiver i) pairs and, per group of rays (as in the forward) 64 at a time,
// mark the rays that a conservative FP32 test cannot rule out (within h_l of
// l), then run the exact FP64 test (the forward's operation sequence) over
// their own marked rays only; each thread sums its pair's contributions in
// registers, one LDS atomic per pair collects them per element, one FP64
// atomic per element and group writes them out.
constexpr int kPRChunk = 256;   // p-p elements per LDS chunk

template <int NB>
__global__ void __launch_bounds__(kNT) k_pp_rays_bwd(const DevTree* __restrict__ TT, Items I,
                                                    const uint32_t* blist, const uint32_t* bscene,
                                                    const uint32_t* noff, const uint32_t* nidx,
                                                    const uint32_t* toff, const uint8_t* active,
                                                    const float* gtppg, Grad Gall) {
  constexpr int RGN = PpRayGroup<NB>::value;
  const int t = threadIdx.x;
  __shared__ RecvInfo recv[kRMax];
  __shared__ uint32_t nrecv_s, s_item;
  __shared__ double rn[RGN][3];
  __shared__ float rnf[RGN][3];
  __shared__ float g[kRMax][RGN][NB];
  __shared__ float ek[kPRChunk][NB], eh[kPRChunk];
  __shared__ int gz;
  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  const Grad G = Gall.at(T);
  const float* gtpp = gtppg + toff[bucket];
  const uint32_t leafb = blist[bucket];
  double c[3];
  leaf_centre(T, leafb, c);
  const uint32_t n0 = noff[bucket], nnear = noff[bucket + 1] - n0;
  const uint32_t* near = nidx + n0;
  const uint2 lk = T.nlink[leafb];
  const int nray = T.nray;
  const int64_t n = T.n;
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
      if (t == 0) gz = 0;
      if (t < kn) {
        const int k = k0 + t;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double na = (k == kd) ? ud[a] : T.ray_n[3 * k + a];
          rn[t][a] = na;
          rnf[t][a] = (float)na;
        }
      }
      __syncthreads();
      int nz = 0;
      for (int q = t; q < nrecv * kn; q += kNT) {
        const int i = q / kn, kq = q % kn;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float v = gtpp[((int64_t)(ract + i) * nray + k0 + kq) * NB + b];
          g[i][kq][b] = v;
          nz |= v != 0.0f;
        }
      }
      if (nz) gz = 1;
      __syncthreads();
      if (!gz) continue;                 // no adjoint on these rays
      for (uint32_t c0 = 0; c0 < nnear; c0 += kPRChunk) {
        const uint32_t cl = min((uint32_t)kPRChunk, nnear - c0);
        for (uint32_t u = t; u < cl; u += kNT) {
#pragma unroll
          for (int b = 0; b < NB; ++b) ek[u][b] = 0.0f;
          eh[u] = 0.0f;
        }
        __syncthreads();
        for (uint32_t pq = t; pq < cl * (uint32_t)nrecv; pq += kNT) {
          const uint32_t u = pq / nrecv;
          const int i = (int)(pq % nrecv);
          const uint32_t l = near[c0 + u];
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
          // column density scale 3m/(pi h^2) and 1/h in FP32 (values, not
          // decisions; no FP64 divisions in this VALU-bound loop)
          const float iv = __builtin_amdgcn_rcpf((float)hl);
          const float sig = (float)(3.0 / kPi) * T.m[l] * iv * iv;
          float kap[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) kap[b] = T.kappa[(int64_t)b * n + l];
          int ka, kb;
          ray_ring_range(T.nside, d0, d1, d2, dd, h2, &ka, &kb);
          const int lo = max(ka - k0, 0), hi = min(kb - k0, kn);
          float ck[NB], gh = 0.0f;
#pragma unroll
          for (int b = 0; b < NB; ++b) ck[b] = 0.0f;
          // the FP32 test over the group's rays in the element's ring range
          // (and the directed ray) first, 64 rays at a time, then the exact
          // test for this lane's candidates only (in ray order)
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
            while (cand) {
              const int kq = s0 + __ffsll((long long)cand) - 1;
              cand &= cand - 1ull;
              const double proj = d0 * rn[kq][0] + d1 * rn[kq][1] + d2 * rn[kq][2];
              const double b2 = dd - proj * proj;
              if (!(proj > 0.0 && b2 < h2)) continue;
              const float bb = __builtin_amdgcn_sqrtf((float)fmax(b2, 0.0));
              const float sg = sig * (1.0f - bb * iv);
              const float dsg = sig * iv * (3.0f * bb * iv - 2.0f);
              float gq = 0.0f;
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                ck[b] += g[i][kq][b] * sg;
                gq += g[i][kq][b] * kap[b];
              }
              gh += gq * dsg;
            }
          }
#pragma unroll
          for (int b = 0; b < NB; ++b)
            if (ck[b] != 0.0f) atomicAdd(&ek[u][b], ck[b]);
          if (gh != 0.0f) atomicAdd(&eh[u], gh);
        }
        __syncthreads();
        for (uint32_t u = t; u < cl; u += kNT) {
          const uint32_t l = near[c0 + u];
#pragma unroll
          for (int b = 0; b < NB; ++b) gadd(&G.gk[(int64_t)b * n + l], (double)ek[u][b]);
          gadd(&G.gh[l], (double)eh[u]);
        }
        __syncthreads();
      }
    }
    ract += (uint32_t)nrecv;
  }
  }
}

// ------------------------------------------------------------- far field
// Sources per LDS window and workgroups per CU of the far-field adjoint:
// the window is sized so that that many workgroups fit in the 160 KiB of
// LDS, and the register budget is held to match (with spilling).  Measured:
// one, two and four bands at four workgroups (two bands with a window of
// 448: 2^21 diffuse 284 -> 224 ms; four bands with 192: batched workload 79
// -> 71 ms), three bands at three (at four, with a window of 320, the clumpy
// scene ran 5% slower); more bands, two (registers limit them anyway).
template <int NB> struct BwdCfg {
  static constexpr int cap = NB == 1 ? 512 : NB == 2 ? 448 : NB == 3 ? 512 : NB == 4 ? 192
                            : NB == 5 ? 512 : NB == 6 ? 448 : NB == 7 ? 320 : 256;
  static constexpr int waves = NB == 3 ? 3 : NB <= 4 ? 4 : 2;
};

// Adjoint of k_far (same workgroup layout).  Per window of sources the cell
// optical depths are recomputed by a first sweep over the hits; the
// (receiver, source) pairs then give, for each term
// L K(r, h_i) exp(-tau_pp - tau_cell r/s) with weight w = w_ib x term:
//   tau_pp adjoint (receiver, ray)  -= w           (LDS atomics)
//   source tau_cell adjoint         -= w r/s       (per source, summed over
//   source s adjoint                += w tau r/s^2  the receivers by shuffles)
//   source luminosity adjoint       += w_ib K e
//   |source - receiver| adjoint     -> source position (merged cells)
//   h_i adjoint                     += w_ib L e dK/dh;
// the background adds its tau_pp and ray-exit adjoints.  A second sweep over
// the hits turns the source tau_cell adjoints into the adjoint of each cell's
// absorption (chord parts inside, whole chords before a source, via suffix
// sums over the ray's sources sorted by distance), of the source distance s
// for sources inside a chord, and of r_pp for chords clipped at the sphere.
template <int NB>
__global__ void __launch_bounds__(kFT, BwdCfg<NB>::waves)
    k_far_bwd(const DevTree* __restrict__ TT, Items I, const uint32_t* blist,
              const uint32_t* bscene, const double* brad, const uint32_t* toff,
              const uint32_t* joff, const uint2* cut, uint32_t cut_cap, const uint32_t* bstat,
              const float* tppall, const float* bgall, const uint8_t* active,
              const double* gJall, const double* jrawall, float* gtppall, Grad Gall,
              const float* kept_tau, const float* kept_tex) {
  constexpr int CAP = BwdCfg<NB>::cap;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

  __shared__ SrcWindow<CAP, NB, false> W;   // suffix adds kept in sgtau
  __shared__ RayGroup RG;
  __shared__ uint32_t sid[CAP];
  __shared__ float sgtau[CAP][NB], sgs[CAP];
  __shared__ float tpp[kRMax][64][NB], gtpp[kRMax][64][NB];
  __shared__ float tex[64][NB], gtex[64][NB];
  __shared__ RecvInfo recv[kRMax];
  __shared__ float gw[kRMax][NB], rinvh[kRMax];
  __shared__ uint32_t nrecv_s, wcnt[kFT / 64], s_item;
  __shared__ double red[kFT / 64][kRMax][NB], redh[kFT / 64][kRMax], redr[kFT / 64];

  for (;;) {
  const uint32_t bucket = next_item(I, &s_item);
  if (bucket == kNoItem) break;
  const DevTree& T = TT[bscene[bucket]];
  const uint8_t* act = active ? active + T.eoff : nullptr;
  const double* gJ = gJall + T.joff;
  const float* bg = bgall ? bgall + T.boff : nullptr;
  const Grad G = Gall.at(T);
  const float* tppg = tppall + toff[bucket];
  float* gtppg = gtppall + toff[bucket];
  const double* jraw = jrawall + joff[bucket];
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
  const bool thick = (T.flags & TREVR_THICK_CORR) != 0u;

  double grpp = 0.0;   // this thread's share of d/d r_pp
  double* const galpha_c = galpha_copy(G);
  double* const gLb_c = gLb_copy(G);
  double* const gcen_c = gcen_copy(G);
  uint32_t ract = 0;
  uint32_t member = lk.x;
  for (;;) {
    const int nrecv = load_receivers(T, act, c, member, lk.x + lk.y, recv, &nrecv_s);
    if (nrecv == 0) break;
    load_receiver_adjoints<NB>(T, gJ, recv, nrecv, gw, rinvh);
    int P2 = 1;
    while (P2 < nrecv) P2 <<= 1;
    const int my_i = t & (P2 - 1);
    const bool has_i = my_i < nrecv;
    const int ii = has_i ? my_i : 0;
    const int per_round = kFT / P2;
    const int my_q = t / P2;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    double ghf = 0.0;

    for (int g = 0; g < ngroups; ++g) {
      const int k0 = 64 * g;
      const int kn = min(64, nray - k0);
      const bool rt = t < kn;
      load_ray_group(T, c, k0, kn, RG);
      for (int q = t; q < nrecv * kn; q += kFT) {
        const int i = q / kn, kq = q % kn;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          tpp[i][kq][b] = tppg[((int64_t)(ract + i) * nray + k0 + kq) * NB + b];
          gtpp[i][kq][b] = 0.0f;
        }
      }
      if (t < kn) {
#pragma unroll
        for (int b = 0; b < NB; ++b) gtex[t][b] = 0.0f;
      }

      for (uint32_t skip = 0;; skip += (uint32_t)CAP) {
        if (t < 64) {
#pragma unroll
          for (int b = 0; b < NB; ++b) tex[t][b] = 0.0f;
        }
        const uint32_t nsg_all = stage_window<CAP, NB>(T, mycut, ncut, c, k0, kn, skip, W, wcnt, sid);
        const uint32_t nsg = min(nsg_all - skip, (uint32_t)CAP);
        for (uint32_t q = t; q < nsg; q += kFT) {
#pragma unroll
          for (int b = 0; b < NB; ++b) sgtau[q][b] = 0.0f;
          sgs[q] = 0.0f;
        }
        uint32_t q0, q1;
        sort_window<CAP, NB>(W, nsg, rt, q0, q1);

        // ---- cell optical depths: recomputed by a first sweep over the hits,
        // or read where the forward kept them (TREVR_KEEP_DEPTHS, the group
        // fitting one window)
        if (kept_tau && skip == 0 && nsg_all <= (uint32_t)KeptCap<NB>::value) {
          const float* src = kept_tau + ((size_t)rel * ngroups + g) * KeptCap<NB>::value * NB;
          for (uint32_t q = t; q < nsg * NB; q += kFT) (&W.tau[0][0])[q] = src[q];
          if (use_bg && t < kn) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
              tex[t][b] = kept_tex[((size_t)rel * nray + k0 + t) * NB + b];
          }
          __syncthreads();
        } else {
          // ---- first sweep: cell optical depths.  Each hit is applied by the
          // thread that found it: sources on its ray inside the chord get the
          // partial length, the nearest source beyond it a suffix add (resolved
          // below along the ray's sources sorted by distance).
          for_each_hit_lane(T, mycut, ncut, c, r, kn, RG,
                            [&](uint32_t node, int kq, double ht0, double ht1, bool) {
            const float len = (float)(ht1 - ht0);
            const float* al = &T.alpha[((int64_t)node * T.nclass + RG.cls[kq]) * NB];
            float av[NB];
  #pragma unroll
            for (int b = 0; b < NB; ++b) {
              av[b] = al[b];
              if (use_bg) atomicAdd(&tex[kq][b], av[b] * len);
            }
            const uint32_t r0 = W.ray_beg[kq], r1 = W.ray_beg[kq + 1];
            uint32_t lo_p = r0, hi_p = r1;
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
              for (int b = 0; b < NB; ++b) atomicAdd(&sgtau[si][b], av[b] * len);
            }
          });
          __syncthreads();
          if (rt) {
            float run[NB];
  #pragma unroll
            for (int b = 0; b < NB; ++b) run[b] = 0.0f;
            for (uint32_t pq = q0; pq < q1; ++pq) {
              const uint32_t si = W.order[pq];
  #pragma unroll
              for (int b = 0; b < NB; ++b) {
                run[b] += sgtau[si][b];
                W.tau[si][b] += run[b];
                sgtau[si][b] = 0.0f;
              }
            }
          }
          __syncthreads();
        }

        // ---- (receiver, source) pairs
        {
          const RecvInfo& ri = recv[ii];
          for (uint32_t q = (uint32_t)my_q; q < nsg; q += (uint32_t)per_round) {
            const float dx = W.rel[q][0] - ri.rel[0];
            const float dy = W.rel[q][1] - ri.rel[1];
            const float dz = W.rel[q][2] - ri.rel[2];
            const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
            const float x = rr * ri.inv_rh;
            const float f = fshape(x);
            const float fd = fshape_d(x);
            const float Kv = f * ri.kfac;
            const float dKdr = fd * ri.inv_rh * ri.kfac;
            const float dKdh = -(2.0f * f + x * fd) * ri.kfac * rinvh[ii];
            const float invs = __builtin_amdgcn_rcpf(W.s[q]);
            const float ratio = rr * invs;
            const int ray = W.ray[q];
            float pL[NB], pt[NB];
            float ps = 0.0f, prr = 0.0f, ph = 0.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const float tau = W.tau[q][b];
              const float tc = (tau > 0.0f) ? tau * ratio : 0.0f;
              const float e = __expf(-(tpp[ii][ray][b] + tc));
              const float Le = W.L[q][b] * e;
              const float LKe = Le * Kv;
              if (has_i) acc[b] += (double)LKe;
              const float gwb = has_i ? gw[ii][b] : 0.0f;
              const float w = gwb * LKe;
              if (w != 0.0f) atomicAdd(&gtpp[ii][ray][b], -w);
              pL[b] = gwb * Kv * e;
              pt[b] = (tau > 0.0f) ? -w * ratio : 0.0f;
              if (tau > 0.0f) {
                ps += w * tc * invs;
                prr -= w * tau * invs;
              }
              prr += gwb * Le * dKdr;
              ph += gwb * Le * dKdh;
            }
            ghf += (double)ph;
            float pp[3] = {0.0f, 0.0f, 0.0f};
            if (rr > 0.0f) {
              const float ir = prr / rr;
              pp[0] = ir * dx;
              pp[1] = ir * dy;
              pp[2] = ir * dz;
            }
            for (int o = 1; o < P2; o <<= 1) {
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                pL[b] += __shfl_xor(pL[b], o);
                pt[b] += __shfl_xor(pt[b], o);
              }
              ps += __shfl_xor(ps, o);
#pragma unroll
              for (int a = 0; a < 3; ++a) pp[a] += __shfl_xor(pp[a], o);
            }
            // every lane of the group now holds the source's totals; the
            // group's lanes share its writes (lane my_i takes outputs my_i,
            // my_i + P2, ...): the NB tau adjoints and the s adjoint to LDS,
            // the NB luminosity adjoints straight to the accumulators, and
            // for merged cells the 3 position adjoints into the source's
            // (no longer read) relative position, added with the s adjoint's
            // part in the flush below
            const uint32_t id = sid[q];
            const bool cell = (id & kSrcCellBit) != 0u;
            const uint32_t node = id & ~kSrcCellBit;
            for (int o = my_i; o <= NB; o += P2) {
              float v = ps;
#pragma unroll
              for (int b = 0; b < NB; ++b)
                if (o == b) v = pt[b];
              if (o < NB) sgtau[q][o] += v;
              else sgs[q] += v;
            }
            const int nglob = cell ? NB + 3 : NB;
            for (int o = my_i; o < nglob; o += P2) {
              float v = 0.0f;
#pragma unroll
              for (int b = 0; b < NB; ++b)
                if (o == b) v = pL[b];
#pragma unroll
              for (int a = 0; a < 3; ++a)
                if (o == NB + a) v = pp[a];
              if (o >= NB) W.rel[q][o - NB] = v;
              else gadd(cell ? &gLb_c[(int64_t)node * NB + o] : &G.gL[(int64_t)o * n + id],
                        (double)v);
            }
          }
          // ---- isotropic background
          if (use_bg && skip == 0) {
            for (int kq = my_q; kq < kn; kq += per_round) {
              float pt[NB];
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const float term = (float)(4.0 * kPi / nray) * bg[b] *
                                   __expf(-(tpp[ii][kq][b] + tex[kq][b]));
                if (has_i) acc[b] += (double)term;
                const float w = has_i ? gw[ii][b] * term : 0.0f;
                if (w != 0.0f) atomicAdd(&gtpp[ii][kq][b], -w);
                pt[b] = -w;
              }
              for (int o = 1; o < P2; o <<= 1) {
#pragma unroll
                for (int b = 0; b < NB; ++b) pt[b] += __shfl_xor(pt[b], o);
              }
              if (my_i == 0) {
#pragma unroll
                for (int b = 0; b < NB; ++b) gtex[kq][b] = pt[b];
              }
            }
          }
        }
        __syncthreads();

        // ---- second sweep: adjoint of the cell optical depths.  W.tau now
        // holds, by sorted position, the suffix sums of the source tau
        // adjoints along each ray.
        if (rt) {
          float run[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) run[b] = 0.0f;
          for (uint32_t pq = q1; pq > q0; --pq) {
            const uint32_t si = W.order[pq - 1];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              run[b] += sgtau[si][b];
              W.tau[pq - 1][b] = run[b];
            }
          }
        }
        __syncthreads();
        const bool bg_here = use_bg && skip == 0;
        for_each_hit_lane(T, mycut, ncut, c, r, kn, RG,
                          [&](uint32_t node, int kq, double ht0, double ht1, bool clipped) {
          const float len = (float)(ht1 - ht0);
          const int cls = RG.cls[kq];
          const float* al = &T.alpha[((int64_t)node * T.nclass + cls) * NB];
          float av[NB], ga[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            av[b] = al[b];
            ga[b] = 0.0f;
          }
          const uint32_t r0 = W.ray_beg[kq], r1 = W.ray_beg[kq + 1];
          uint32_t lo_p = r0, hi_p = r1;
          while (lo_p < hi_p) {
            const uint32_t mid = (lo_p + hi_p) >> 1;
            if ((double)W.s[W.order[mid]] > ht0) hi_p = mid; else lo_p = mid + 1;
          }
          const uint32_t first = lo_p;
          uint32_t pq = first;
          for (; pq < r1; ++pq) {
            const uint32_t si = W.order[pq];
            const double sq = (double)W.s[si];
            if (!(sq < ht1)) break;
            const float part = (float)(sq - ht0);
            float gs = 0.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              ga[b] += sgtau[si][b] * part;
              gs += sgtau[si][b] * av[b];
            }
            if (gs != 0.0f) atomicAdd(&sgs[si], gs);
          }
          if (pq < r1) {
#pragma unroll
            for (int b = 0; b < NB; ++b) ga[b] += len * W.tau[pq][b];
          }
          float gr = 0.0f;
          if (clipped && first < r1) {
#pragma unroll
            for (int b = 0; b < NB; ++b) gr += av[b] * W.tau[first][b];
          }
          if (bg_here) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              ga[b] += len * gtex[kq][b];
              if (clipped) gr += av[b] * gtex[kq][b];
            }
          }
          grpp -= (double)gr;
          double* dst = &galpha_c[((int64_t)node * T.nclass + cls) * NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) gadd(&dst[b], (double)ga[b]);
        });
        __syncthreads();

        // ---- flush the source adjoints
        for (uint32_t q = t; q < nsg; q += kFT) {   // merged cells: position adjoints
          const uint32_t id = sid[q];
          if (id & kSrcCellBit) {
            const uint32_t node = id & ~kSrcCellBit;
            const int ray = W.ray[q];
            const double gs = W.s[q] != 0.0f ? (double)sgs[q] : 0.0;   // s = (p - c).n
#pragma unroll
            for (int a = 0; a < 3; ++a)
              gadd(&gcen_c[(int64_t)node * 4 + a], (double)W.rel[q][a] + gs * RG.n[ray][a]);
          }
        }
        __syncthreads();
        if (nsg_all <= skip + (uint32_t)CAP) break;
      }
      // p-p column adjoints of this ray group
      for (int q = t; q < nrecv * kn; q += kFT) {
        const int i = q / kn, kq = q % kn;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          gtppg[((int64_t)(ract + i) * nray + k0 + kq) * NB + b] = gtpp[i][kq][b];
      }
      __syncthreads();
    }

    // ---- per receiver: raw J (p-p + far), the thick-element factor
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = acc[b];
      for (int o = 32; o >= P2 && o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane < P2 && lane < nrecv) red[wv][lane][b] = v;
    }
    {
      double v = ghf;
      for (int o = 32; o >= P2 && o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane < P2 && lane < nrecv) redh[wv][lane] = v;
    }
    __syncthreads();
    if (t < nrecv * NB) {
      const int i = t / NB, b = t % NB;
      double v = 0.0;
      for (int w = 0; w < kFT / 64; ++w) v += red[w][i][b];
      if (thick) {
        const uint32_t sl = recv[i].slot;
        const double Jr = jraw[(int64_t)(ract + i) * NB + b] + v;
        const double kap = (double)T.kappa[(int64_t)b * n + sl], rho = (double)T.rho[sl];
        const double h = recv[i].h;
        const double gC = gJ[(int64_t)b * n + T.perm[sl]] * Jr * thick_dC(kap * rho * h);
        gadd(&G.gk[(int64_t)b * n + sl], gC * rho * h);
        gadd(&G.gr[sl], gC * kap * h);
        gadd(&G.gh[sl], gC * kap * rho);
      }
    }
    if (t < nrecv) {
      double v = 0.0;
      for (int w = 0; w < kFT / 64; ++w) v += redh[w][t];
      gadd(&G.gh[recv[t].slot], v);
    }
    __syncthreads();
    ract += (uint32_t)nrecv;
  }
  // ---- r_pp adjoint of the bucket
  const double v = wave_sum(grpp);
  if (lane == 0) redr[wv] = v;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < kFT / 64; ++w) s += redr[w];
    G.grpp[bucket] = s;
  }
  }
}

// ---------------------------------------------------------- p-p radius
// The p-p radius is a maximum (Section 2.4): of rpp_min and the members'
// reach |x_s - c| + h_s, then of the beam rule h_j / w while the sphere
// grows.  Its adjoint goes to the h of the element that set it: the first
// in sorted order among equal values; for the beam rule the setup recorded
// that element (inside the sphere of the round that set the final radius).
// One thread per bucket (the work per bucket is a few loads).
__global__ void k_rpp_bwd(const DevTree* __restrict__ TT, const uint32_t* nbp,
                          const uint32_t* blist, const uint32_t* bscene, const double* bprev,
                          const uint32_t* barg, Grad Gall) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *nbp) return;
  const double g = Gall.grpp[b];
  if (g == 0.0) return;
  const DevTree& T = TT[bscene[b]];
  if (!(T.flags & TREVR_NEAR_FIELD)) return;
  const Grad G = Gall.at(T);
  if (bprev[b] >= 0.0) {   // the beam rule of the last growth
    if (barg[b] != 0xFFFFFFFFu) gadd(&G.gh[barg[b]], g / T.wbeam);
    return;
  }
  // never grew: the largest member reach |x - c| + h, first slot attaining
  // it, unless rpp_min was larger
  double c[3];
  leaf_centre(T, blist[b], c);
  const uint2 lk = T.nlink[blist[b]];
  double rm = -INFINITY;
  uint32_t arg = 0xFFFFFFFFu;
  for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) {
    const double v = sqrt(dist2_pt3((double)T.x[s], (double)T.y[s], (double)T.z[s], c)) + T.h[s];
    if (v > rm) {
      rm = v;
      arg = s;
    }
  }
  if (rm > T.rpp_min && arg != 0xFFFFFFFFu) gadd(&G.gh[arg], g);
}

// ------------------------------------------------------------ the tree
// Centre adjoint -> (u, v): the centre c = sum(L_s x_s)/L of a node moves
// by (x_s - c)/L per unit of any band of L_s, so element s collects
// u.x_s - v over its ancestors with u = dE/dc / L, v = u.c.
__global__ void k_cen_prep(const DevTree* __restrict__ TT, Grad Gall) {
  const DevTree& T = TT[blockIdx.y];
  const Grad G = Gall.at(T);
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= T.num_nodes) return;
  const double4 cn = T.cen[p];
  double* g = G.gcen + 4 * p;
  if (cn.w > 0.0) {
    const double u0 = g[0] / cn.w, u1 = g[1] / cn.w, u2 = g[2] / cn.w;
    g[0] = u0;
    g[1] = u1;
    g[2] = u2;
    g[3] = u0 * cn.x + u1 * cn.y + u2 * cn.z;
  } else {
    g[0] = g[1] = g[2] = g[3] = 0.0;
  }
}

// One level of internal nodes (top-down), one thread per (node, class):
// the transmission average alpha = combine_s(alpha_c0, alpha_c1) grown
// through the empty prefix boxes (Section 2.6) passes its adjoint to the
// children; class 0 also passes the luminosity and centre adjoints.
__global__ void k_tree_bwd(const DevTree* __restrict__ TT, int depth, Grad Gall) {
  const DevTree& T = TT[blockIdx.y];
  if (depth >= T.depth) return;
  const Grad G = Gall.at(T);
  const uint2 lv = T.levels[depth];
  const uint32_t lb = lv.x, le = lv.y;
  const int B = T.B, nclass = T.nclass;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)(le - lb) * nclass) return;
  const uint32_t i = lb + (uint32_t)(gid / nclass);
  const int c = (int)(gid % nclass);
  const int s = T.b_split[i];
  if (s < 0) return;
  const uint32_t p = T.b_pre[i], p0 = p + 1u, p1 = T.nlink[p].x;
  const int l = T.b_lown[i];
  const double L = T.hdr[3];
  for (int b = 0; b < B; ++b) {
    const double g = G.galpha[((int64_t)p * nclass + c) * B + b];
    if (g == 0.0) continue;
    double d1, d2;
    double D = 1.0;
    if (T.flags & TREVR_ABSORPTION_AVG) {
      d1 = d2 = 0.5;
      for (int mm = s - 1; mm >= l; --mm) D *= 0.5;
    } else {
      double A = combine64_d(&T.geom[((int64_t)s * nclass + c) * 3], L,
                             T.alpha64[((int64_t)p0 * nclass + c) * B + b],
                             T.alpha64[((int64_t)p1 * nclass + c) * B + b], &d1, &d2);
      for (int mm = s - 1; mm >= l; --mm) {
        double e1, e2;
        A = combine64_d(&T.geom[((int64_t)mm * nclass + c) * 3], L, A, 0.0, &e1, &e2);
        D *= e1;
      }
    }
    G.galpha[((int64_t)p0 * nclass + c) * B + b] += g * D * d1;
    G.galpha[((int64_t)p1 * nclass + c) * B + b] += g * D * d2;
  }
  if (c == 0) {
    for (int b = 0; b < B; ++b) {
      const double v = G.gLb[(int64_t)p * B + b];
      G.gLb[(int64_t)p0 * B + b] += v;
      G.gLb[(int64_t)p1 * B + b] += v;
    }
    for (int a = 0; a < 4; ++a) {
      const double v = G.gcen[4 * (int64_t)p + a];
      G.gcen[4 * (int64_t)p0 + a] += v;
      G.gcen[4 * (int64_t)p1 + a] += v;
    }
  }
}

// Buckets: alpha_b = sum(kappa_b m)/sum(m/rho) for every class, so
// dkappa_bs += A_b m_s/V and drho_s += sum_b A_b alpha_b m_s/(rho_s^2 V)
// with A_b the adjoint summed over classes; luminosities collect the
// accumulated (Lb, centre) adjoints of the path to the root.
__global__ void k_leaf_bwd(const DevTree* __restrict__ TT, Grad Gall) {
  const DevTree& T = TT[blockIdx.y];
  const Grad G = Gall.at(T);
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= T.num_nodes) return;
  if (!(T.nk[p].w & META_LEAF)) return;
  const int B = T.B, nclass = T.nclass;
  const int64_t n = T.n;
  const uint2 lk = T.nlink[p];
  double A[kMaxBands], ab[kMaxBands];
  for (int b = 0; b < B; ++b) {
    double s = 0.0;
    for (int c = 0; c < nclass; ++c) s += G.galpha[((int64_t)p * nclass + c) * B + b];
    A[b] = s;
    ab[b] = T.alpha64[(int64_t)p * nclass * B + b];
  }
  double vol = 0.0;
  for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) vol += (double)T.m[s] / (double)T.rho[s];
  const double* gc = G.gcen + 4 * p;
  for (uint32_t s = lk.x; s < lk.x + lk.y; ++s) {
    const double ms = (double)T.m[s], rs = (double)T.rho[s];
    double gr = 0.0;
    for (int b = 0; b < B; ++b) {
      G.gk[(int64_t)b * n + s] += A[b] * ms / vol;
      gr += A[b] * ab[b];
    }
    G.gr[s] += gr * ms / (rs * rs * vol);
    const double gl = gc[0] * (double)T.x[s] + gc[1] * (double)T.y[s] + gc[2] * (double)T.z[s] - gc[3];
    for (int b = 0; b < B; ++b) G.gL[(int64_t)b * n + s] += G.gLb[p * B + b] + gl;
  }
}

// h = (m/rho)^(1/3): dh/drho = -h/(3 rho).  Gradients to input order.
__global__ void k_grad_out(const DevTree* __restrict__ TT, Grad Gall, double* gLall,
                           double* gkall, double* grhoall) {
  const DevTree& T = TT[blockIdx.y];
  const Grad G = Gall.at(T);
  double* gL = gLall + T.joff;
  double* gk = gkall + T.joff;
  double* grho = grhoall + T.eoff;
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= T.n) return;
  const int64_t n = T.n;
  const uint32_t i = T.perm[s];
  grho[i] = G.gr[s] - G.gh[s] * T.h[s] / (3.0 * (double)T.rho[s]);
  for (int b = 0; b < T.B; ++b) {
    gL[(int64_t)b * n + i] = G.gL[(int64_t)b * n + s];
    gk[(int64_t)b * n + i] = G.gk[(int64_t)b * n + s];
  }
}

// Sum the copies of an accumulator into the first.
__global__ void k_sum_copies(double* a, int64_t per, uint32_t copies) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= per) return;
  double s = a[i];
  for (uint32_t k = 1; k < copies; ++k) s += a[(int64_t)k * per + i];
  a[i] = s;
}

// ============================================================ host side
static unsigned grid_of(int64_t work, int threads) {
  return (unsigned)std::max<int64_t>(1, (work + threads - 1) / threads);
}

Grad carve_grad(Carve& cv, const GradDims& d) {
  Grad g{};
  g.gL = cv.take<double>(d.jn);
  g.gk = cv.take<double>(d.jn);
  g.gh = cv.take<double>(d.n);
  g.gr = cv.take<double>(d.n);
  // copies of the far-field accumulators within a budget of 256 MiB each
  const size_t budget = (size_t)256 << 20;
  g.na = d.alpha;
  g.ns = d.nodesB;
  g.nc = 4 * d.nodes;
  g.ka = 1;
  while (g.ka < 8 && (size_t)(2 * g.ka) * g.na * sizeof(double) <= budget) g.ka *= 2;
  g.ks = 1;
  while (g.ks < 16 && (size_t)(2 * g.ks) * (g.ns + g.nc) * sizeof(double) <= budget) g.ks *= 2;
  g.galpha = cv.take<double>((size_t)g.ka * g.na);
  g.gLb = cv.take<double>((size_t)g.ks * g.ns);
  g.gcen = cv.take<double>((size_t)g.ks * g.nc);
  g.grpp = cv.take<double>(std::max<int64_t>(d.leaves, 1));
  return g;
}

#define TREVR_LAUNCH_CHECK(what)                                               \
  do {                                                                         \
    if ((rc = hip_check(hipGetLastError(), what)) != TREVR_OK) return rc;      \
  } while (0)

template <int NB>
static trevr_status bwd_items_nb(const Launch& L, const Scratch& S, const BwdArgs& a,
                                 const Items& I, uint64_t count, uint32_t cap,
                                 Prof* prof) {
  trevr_status rc;
  hipEvent_t e0 = prof_begin(prof, L.st);
  {
    const Items Ii{I.lo, I.hi, I.rng, S.q + 2 * Q_PPS_BWD};
    const void* fn = (const void*)&k_pp_src_bwd<NB>;
    k_pp_src_bwd<NB><<<persistent_grid(fn, kNT, count, L.cfg.grid_div), kNT, 0, L.st>>>(
        L.TT, Ii, S.blist, S.bscene, S.ncnt, S.nlumc, S.nidx, S.jcnt, S.pcnt, S.ptau, a.active,
        a.gJ, a.G, a.jraw, S.jlog);
    TREVR_LAUNCH_CHECK("k_pp_src_bwd");
  }
  const size_t recorded = prof ? prof->pending.size() : 0;
  prof_end(prof, L.st, TREVR_PROF_ADJ_NEAR, e0);
  if (prof && prof->pending.size() == recorded + 1)   // the same span, p-p source adjoint alone
    prof->pending.push_back({TREVR_PROF_ADJ_PP_SRC, prof->pending.back().second});
  hipEvent_t e1 = prof_begin(prof, L.st);
  {
    const Items Ii{I.lo, I.hi, I.rng, S.q + 2 * Q_FAR_BWD};
    const void* fn = (const void*)&k_far_bwd<NB>;
    k_far_bwd<NB><<<persistent_grid(fn, kFT, count, L.cfg.grid_div), kFT, 0, L.st>>>(
        L.TT, Ii, S.blist, S.bscene, S.brad, S.tcnt, S.jcnt, S.cut, cap, S.bstat, S.tpp, a.bg,
        a.active, a.gJ, a.jraw, a.gtpp, a.G, a.kept_tau, a.kept_tex);
    TREVR_LAUNCH_CHECK("k_far_bwd");
  }
  prof_end(prof, L.st, TREVR_PROF_ADJ_REDUCE, e1);
  hipEvent_t e2 = prof_begin(prof, L.st);
  {
    const Items Ii{I.lo, I.hi, I.rng, S.q + 2 * Q_PPR_BWD};
    const void* fn = (const void*)&k_pp_rays_bwd<NB>;
    k_pp_rays_bwd<NB><<<persistent_grid(fn, kNT, count, L.cfg.grid_div), kNT, 0, L.st>>>(
        L.TT, Ii, S.blist, S.bscene, S.ncnt, S.nidx, S.tcnt, a.active, a.gtpp, a.G);
    TREVR_LAUNCH_CHECK("k_pp_rays_bwd");
  }
  prof_end(prof, L.st, TREVR_PROF_ADJ_NEAR, e2);
  return rc;
}

trevr_status bwd_items(const Launch& L, int B, const Scratch& S, const BwdArgs& a,
                       const Items& I, uint64_t count, uint32_t cap, Prof* prof) {
  switch (B) {
    case 1: return bwd_items_nb<1>(L, S, a, I, count, cap, prof);
    case 2: return bwd_items_nb<2>(L, S, a, I, count, cap, prof);
    case 3: return bwd_items_nb<3>(L, S, a, I, count, cap, prof);
    case 4: return bwd_items_nb<4>(L, S, a, I, count, cap, prof);
    case 5: return bwd_items_nb<5>(L, S, a, I, count, cap, prof);
    case 6: return bwd_items_nb<6>(L, S, a, I, count, cap, prof);
    case 7: return bwd_items_nb<7>(L, S, a, I, count, cap, prof);
    case 8: return bwd_items_nb<8>(L, S, a, I, count, cap, prof);
    case 9: return bwd_items_nb<9>(L, S, a, I, count, cap, prof);
    case 10: return bwd_items_nb<10>(L, S, a, I, count, cap, prof);
    case 11: return bwd_items_nb<11>(L, S, a, I, count, cap, prof);
    case 12: return bwd_items_nb<12>(L, S, a, I, count, cap, prof);
    case 13: return bwd_items_nb<13>(L, S, a, I, count, cap, prof);
    case 14: return bwd_items_nb<14>(L, S, a, I, count, cap, prof);
    case 15: return bwd_items_nb<15>(L, S, a, I, count, cap, prof);
    default: return bwd_items_nb<16>(L, S, a, I, count, cap, prof);
  }
}

trevr_status bwd_tree_pass(const Launch& L, const Scratch& S, const Grad& G,
                           const std::vector<int64_t>& level_work, double* gL, double* gk,
                           double* grho) {
  hipStream_t st = L.st;
  trevr_status rc;
  k_rpp_bwd<<<grid_of(L.leaves, 256), 256, 0, st>>>(L.TT, S.rng + 1, S.blist, S.bscene,
                                                     S.bprev, S.barg, G);
  TREVR_LAUNCH_CHECK("k_rpp_bwd");
  if (G.ka > 1) {
    k_sum_copies<<<grid_of(G.na, 256), 256, 0, st>>>(G.galpha, G.na, G.ka);
    TREVR_LAUNCH_CHECK("k_sum_copies");
  }
  if (G.ks > 1) {
    k_sum_copies<<<grid_of(G.ns, 256), 256, 0, st>>>(G.gLb, G.ns, G.ks);
    TREVR_LAUNCH_CHECK("k_sum_copies");
    k_sum_copies<<<grid_of(G.nc, 256), 256, 0, st>>>(G.gcen, G.nc, G.ks);
    TREVR_LAUNCH_CHECK("k_sum_copies");
  }
  const unsigned S_ = (unsigned)L.S;
  k_cen_prep<<<dim3(grid_of(L.max_nodes, 256), S_), 256, 0, st>>>(L.TT, G);
  TREVR_LAUNCH_CHECK("k_cen_prep");
  for (size_t d = 0; d < level_work.size(); ++d) {
    k_tree_bwd<<<dim3(grid_of(level_work[d], 128), S_), 128, 0, st>>>(L.TT, (int)d, G);
    TREVR_LAUNCH_CHECK("k_tree_bwd");
  }
  k_leaf_bwd<<<dim3(grid_of(L.max_nodes, 128), S_), 128, 0, st>>>(L.TT, G);
  TREVR_LAUNCH_CHECK("k_leaf_bwd");
  k_grad_out<<<dim3(grid_of(L.max_n, 256), S_), 256, 0, st>>>(L.TT, G, gL, gk, grho);
  TREVR_LAUNCH_CHECK("k_grad_out");
  return TREVR_OK;
}

// Scratch of the backward: the forward's layout (fixed part, p-p lists,
// p-p columns, pair depths, kept depths), then the p-p column adjoints, the
// raw J per receiver and the gradient accumulators.  When the scratch still
// holds the state of a compute_J on this tree for the same active set (same
// buffer, not written by any call since, equal fingerprint), its bucket
// setup, p-p lists, p-p columns and (with a single batch) cut lists are used
// as they are.
trevr_status compute_J_backward_impl(trevr_tree* T, const uint8_t* active, const float* bg,
                                     const double* gJ, double* gL, double* gkappa, double* grho,
                                     void* scratch, size_t scratch_bytes) {
  hipStream_t st = T->stream;
  Scratch S = carve_scratch(scratch, T->num_leaves, default_cut_entries(T->num_leaves));
  S.stage_cap = std::min(S.stage_cap, T->stage_limit & ~63u);
  if (scratch_bytes < S.fixed) {
    T->scratch_needed = S.fixed;
    return set_error(TREVR_E_CAPACITY, "scratch smaller than its fixed part");
  }
  trevr_status rc;
  hipEvent_t ev_setup = prof_begin(T);
  bool reuse = false;
  if (T->fwd.valid && T->fwd.scratch == scratch && scratch_unchanged(scratch, T->fwd.epoch)) {
    uint64_t h = 0;
    if ((rc = active_hash(T, active, S.ahash + 1, &h)) != TREVR_OK) return rc;
    reuse = h == T->fwd.hash;
  }
  uint64_t hash = T->fwd.hash;
  uint32_t nb = 0;
  uint64_t tot[TOT_N] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (reuse) {
    nb = T->fwd.nb;
    tot[TOT_NEAR] = T->fwd.near_total;
    tot[TOT_TPP] = T->fwd.tpp_total;
    tot[TOT_PTAU] = T->fwd.ptau_total;
    tot[TOT_JRAW] = T->fwd.jraw_total;
    // the work-queue counters of the forward are zero after its launches
  } else {
    T->fwd.valid = false;
    if ((rc = bucket_setup(T, active, S, &nb, tot, &hash)) != TREVR_OK) return rc;
  }
  Carve dyn((char*)scratch + S.fixed);
  S.nidx = dyn.take<uint32_t>(tot[TOT_NEAR]);
  S.tpp = dyn.take<float>(tot[TOT_TPP]);
  S.ptau = dyn.take<float>(tot[TOT_PTAU]);
  take_kept(T, S, dyn, nb);
  // the forward's far-source optical depths apply to its own (single) batch
  const bool use_kept = reuse && T->fwd.kept && S.kept_tau != nullptr;
  BwdArgs a{};
  a.active = active;
  a.bg = bg;
  a.gJ = gJ;
  a.kept_tau = use_kept ? S.kept_tau : nullptr;
  a.kept_tex = use_kept ? S.kept_tex : nullptr;
  a.gtpp = dyn.take<float>(tot[TOT_TPP]);
  a.jraw = dyn.take<double>(tot[TOT_JRAW]);
  const size_t gbeg = (S.fixed + dyn.off + 255) & ~(size_t)255;
  Carve gcv((char*)scratch + gbeg);
  GradDims dims{T->B * T->n, T->n, T->num_nodes, T->num_nodes * T->B,
                T->num_nodes * T->nclass * T->B, T->num_leaves};
  a.G = carve_grad(gcv, dims);
  const size_t gbytes = (gcv.off + 255) & ~(size_t)255;
  const size_t need = gbeg + gbytes + 256;
  T->scratch_needed = need;
  if (scratch_bytes < need) return set_error(TREVR_E_CAPACITY, "scratch too small for the adjoint");
  const uint64_t epoch = scratch_mark(scratch);
  if ((rc = zero_words(st, (char*)scratch + gbeg, gbytes / 4)) != TREVR_OK) return rc;
  if (!reuse && (rc = near_fill(tree_launch(T), S)) != TREVR_OK) return rc;
  prof_end(T, TREVR_PROF_SETUP, ev_setup);
  auto run = [&](uint32_t s0, uint32_t scnt, uint32_t cap) -> trevr_status {
    trevr_status r;
    const Launch L = tree_launch(T);
    if (!reuse) {   // the forward's p-p columns and pair optical depths
      hipEvent_t ev_near = prof_begin(T);
      if ((r = launch_pp_rays(L, T->B, S, host_items(S, Q_PPR, s0, scnt), scnt, active)) !=
          TREVR_OK)
        return r;
      if ((r = launch_pp_src(L, T->B, S, host_items(S, Q_PPS, s0, scnt), scnt, active,
                             nullptr)) != TREVR_OK)
        return r;
      prof_end(T, TREVR_PROF_NEAR, ev_near);
    }
    return bwd_items(L, T->B, S, a, Items{s0, s0 + scnt, nullptr, nullptr}, scnt, cap,
                     &T->prof);
  };
  bool whole = reuse && T->fwd.cuts_kept;
  if (whole) {   // one batch, whose cut lists the forward left in place
    if (nb > 0 && (rc = run(0, nb, T->fwd.cut_stride)) != TREVR_OK) return rc;
  } else {
    whole = true;
    for (uint32_t b0 = 0; b0 < nb; b0 += kBatch) {
      const uint32_t cnt = std::min<uint32_t>(kBatch, nb - b0);
      bool w = true;
      if ((rc = walk_batch(T, S, b0, cnt, run, &w)) != TREVR_OK) return rc;
      whole = whole && w;
    }
  }
  hipEvent_t ev_tree = prof_begin(T);
  std::vector<int64_t> level_work;
  for (const auto& lv : T->levels) level_work.push_back((int64_t)(lv.second - lv.first) * T->nclass);
  if ((rc = bwd_tree_pass(tree_launch(T), S, a.G, level_work, gL, gkappa, grho)) != TREVR_OK)
    return rc;
  prof_end(T, TREVR_PROF_ADJ_TREE, ev_tree);
  T->fwd = FwdState{true, scratch, epoch, hash, nb, tot[TOT_NEAR], tot[TOT_TPP], tot[TOT_PTAU],
                    tot[TOT_JRAW], nb <= kBatch && whole, T->cut_default, use_kept};
  return TREVR_OK;
}
#undef TREVR_LAUNCH_CHECK

}  // namespace trevr
