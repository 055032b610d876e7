// Host-only sanitizer run of the FP64 oracle (test infrastructure): this file
// is compiled together with oracle/trevr_oracle.cpp as one translation unit
// under AddressSanitizer and UndefinedBehaviorSanitizer (static runtimes), and
// drives the oracle's C ABI on small synthetic scenes: every option flag,
// one to ten bands, N_side 1-4, an active subset, the forward-mode
// derivative, the complex source tables and the unit functions.  It prints
// one line per case; any sanitizer report aborts with a nonzero status.
#include "../oracle/trevr_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {
// 64-bit linear congruential generator (Knuth's MMIX constants), top 53 bits
struct Lcg {
  uint64_t s;
  double next() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

int run_case(int n, int nside, int B, uint32_t flags, int leaf, double active_frac, uint64_t seed) {
  Lcg g{seed};
  std::vector<double> x(n), y(n), z(n), m(n), rho(n), kap((size_t)B * n), lum((size_t)B * n);
  std::vector<uint8_t> act(n);
  for (int i = 0; i < n; ++i) {
    x[i] = g.next();
    y[i] = g.next();
    z[i] = g.next();
    rho[i] = 0.5 + 2.0 * g.next();
    m[i] = rho[i] * std::pow(0.08 + 0.1 * g.next(), 3.0);
    act[i] = g.next() < active_frac ? 1 : 0;
    for (int b = 0; b < B; ++b) {
      kap[(size_t)b * n + i] = (b + 1) * (0.5 + g.next());
      lum[(size_t)b * n + i] = (i % 7 == 0) ? 1.0 + g.next() : 0.0;
    }
  }
  act[0] = 1;
  Params p{};
  p.nside = nside;
  p.leaf_size = leaf;
  p.n_bands = B;
  p.flags = flags;
  p.theta = 0.75;
  p.rpp_min = 0.0;
  p.target[0] = 0.3;
  p.target[1] = 0.6;
  p.target[2] = 0.4;
  std::vector<double> bg(B, 0.01);
  std::vector<double> J((size_t)B * n, 0.0), dJ((size_t)B * n, 0.0);
  std::vector<int64_t> cnt(C_N, 0);
  void* h = ora_build(&p, n, x.data(), y.data(), z.data(), m.data(), rho.data(), kap.data(),
                      lum.data());
  const int64_t nn = ora_num_nodes(h);
  std::vector<double> info((size_t)6 * nn);
  ora_compute_J(h, act.data(), bg.data(), J.data(), cnt.data(), info.data(), 2);
  if (flags & F_CPLX) {
    const int K = 12 * nside * nside;
    std::vector<double> cd((size_t)nn * K), ca((size_t)nn * K * B);
    std::vector<int32_t> anti(K);
    ora_complex(h, cd.data(), ca.data(), anti.data());
  }
  ora_free(h);
  std::vector<double> tL((size_t)B * n), tk((size_t)B * n), tr(n);
  for (size_t i = 0; i < tL.size(); ++i) {
    tL[i] = g.next() - 0.5;
    tk[i] = g.next() - 0.5;
  }
  for (int i = 0; i < n; ++i) tr[i] = g.next() - 0.5;
  std::fill(J.begin(), J.end(), 0.0);
  ora_jvp(&p, n, x.data(), y.data(), z.data(), m.data(), rho.data(), kap.data(), lum.data(),
          act.data(), bg.data(), tL.data(), tk.data(), tr.data(), J.data(), dJ.data(), cnt.data(), 2);
  double s = 0.0;
  for (double v : J) s += v;
  std::printf("n %d nside %d bands %d flags %u: segments %lld, sum J %.6e\n", n, nside, B, flags,
              (long long)cnt[C_SEG], s);
  return std::isfinite(s) ? 0 : 1;
}
}  // namespace

int main() {
  int bad = 0;
  bad |= run_case(300, 1, 1, F_NEAR | F_THICK, 8, 1.0, 1);
  bad |= run_case(400, 2, 3, F_NEAR | F_THICK | F_BG, 8, 0.3, 2);
  bad |= run_case(400, 2, 2, F_NEAR | F_AVG | F_DIRECTED, 12, 0.5, 3);
  bad |= run_case(300, 2, 2, F_NEAR | F_CPLX, 8, 1.0, 4);
  bad |= run_case(200, 4, 10, F_NEAR | F_BG, 8, 0.2, 5);
  bad |= run_case(64, 1, 1, 0u, 1, 1.0, 6);
  // unit functions
  std::vector<double> cen(3 * 48);
  ora_healpix_centres(2, cen.data());
  std::vector<int32_t> pix(48);
  ora_healpix_pixel(2, 48, cen.data(), pix.data());
  for (int k = 0; k < 48; ++k) bad |= pix[k] != k;
  bad |= !std::isfinite(ora_kernel_K(0.3, 0.1)) || !std::isfinite(ora_thick_C(0.5));
  std::printf("unit functions: %s\n", bad ? "FAIL" : "ok");
  return bad;
}
