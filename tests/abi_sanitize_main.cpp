// Host-side sanitizer run of the C ABI (test infrastructure): linked against
// a build of the library whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer, it drives every path that runs without a GPU:
// workspace sizing for all option flags, band counts and N_side values,
// forest sizing, argument validation (bad sizes, parameters, pointers and
// handles), status strings and the last-error text.  Exit status 0 when
// every call returned what the header documents; any sanitizer report
// aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../include/trevr2.h"

namespace {
int failures = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++failures;
  }
}

trevr_params params(int nside, int B, uint32_t flags) {
  trevr_params p{};
  p.nside = nside;
  p.leaf_size = 8;
  p.n_bands = B;
  p.flags = flags;
  p.theta = 0.75;
  p.rpp_min = 0.0;
  p.target[0] = 0.5;
  p.target[1] = 0.5;
  p.target[2] = 0.5;
  return p;
}
}  // namespace

int main() {
  // sizing across options
  const uint32_t flag_sets[] = {0u, 1u | 2u, 1u | 2u | 4u, 2u | 8u, 2u | 16u, 2u | 32u, 2u | 64u};
  for (int nside = 1; nside <= 16; nside *= 2)
    for (int B = 1; B <= 16; B += 5)
      for (uint32_t f : flag_sets) {
        trevr_params p = params(nside, B, f);
        size_t tb = 0, sb = 0;
        expect(trevr_workspace_bytes(&p, 5000, &tb, &sb) == TREVR_OK && tb > 0 && sb > 0,
               "workspace sizing");
      }
  // invalid parameters and sizes
  {
    trevr_params bad[] = {params(3, 1, 2u), params(0, 1, 2u), params(32, 1, 2u), params(2, 0, 2u),
                          params(2, 17, 2u), params(2, 1, 128u)};
    for (auto& p : bad) {
      size_t tb, sb;
      expect(trevr_workspace_bytes(&p, 100, &tb, &sb) == TREVR_E_INVALID, "invalid params");
    }
    trevr_params p = params(2, 1, 32u);
    p.target[0] = NAN;
    size_t tb, sb;
    expect(trevr_workspace_bytes(&p, 100, &tb, &sb) == TREVR_E_INVALID, "directed without target");
    p = params(2, 1, 2u);
    p.theta = -1.0;
    expect(trevr_workspace_bytes(&p, 100, &tb, &sb) == TREVR_E_INVALID, "negative theta");
    p = params(2, 1, 2u);
    for (int64_t n : {(int64_t)0, (int64_t)-5, (int64_t)1 << 31})
      expect(trevr_workspace_bytes(&p, n, &tb, &sb) == TREVR_E_INVALID, "bad n");
    expect(trevr_workspace_bytes(nullptr, 100, &tb, &sb) == TREVR_E_INVALID, "null params");
    trevr_tree* t = nullptr;
    expect(trevr_build_tree(&p, 1000, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, 0, nullptr, &t) == TREVR_E_INVALID && !t,
           "build with null inputs");
  }
  // unknown handles
  {
    trevr_tree* bogus = reinterpret_cast<trevr_tree*>(0x12345678);
    trevr_counters c;
    expect(trevr_check(bogus) == TREVR_E_STATE, "check unknown tree");
    expect(trevr_get_counters(bogus, &c) == TREVR_E_STATE, "counters unknown tree");
    expect(trevr_tree_tune(bogus, 0, 1) == TREVR_E_STATE, "tune unknown tree");
    expect(trevr_tree_destroy(bogus) == TREVR_E_STATE, "destroy unknown tree");
    trevr_forest* fb = reinterpret_cast<trevr_forest*>(0x87654321);
    size_t sz;
    expect(trevr_forest_check(fb) == TREVR_E_STATE, "check unknown forest");
    expect(trevr_forest_plan_bytes(fb, &sz) == TREVR_E_STATE, "plan bytes unknown forest");
    expect(trevr_forest_job_log(fb, 1u << 20) == TREVR_E_STATE, "job log unknown forest");
    expect(trevr_forest_destroy(fb) == TREVR_E_STATE, "destroy unknown forest");
  }
  // forest sizing and validation
  {
    std::vector<trevr_params> P = {params(1, 1, 3u), params(2, 3, 7u), params(4, 2, 2u | 8u)};
    const int64_t ok[4] = {0, 100, 350, 1000};
    size_t sz = 0;
    expect(trevr_forest_workspace_bytes(P.data(), 3, ok, &sz) == TREVR_OK && sz > 0,
           "forest sizing");
    const int64_t bad1[4] = {0, 100, 100, 1000}, bad2[4] = {5, 100, 350, 1000};
    expect(trevr_forest_workspace_bytes(P.data(), 3, bad1, &sz) == TREVR_E_INVALID,
           "forest empty scene");
    expect(trevr_forest_workspace_bytes(P.data(), 3, bad2, &sz) == TREVR_E_INVALID,
           "forest offsets not from 0");
    expect(trevr_forest_workspace_bytes(P.data(), 0, ok, &sz) == TREVR_E_INVALID,
           "forest of no scene");
  }
  for (int s = 0; s < 6; ++s) expect(trevr_status_string((trevr_status)s)[0] != '\0', "status");
  expect(trevr_last_error() != nullptr, "last error");
  std::printf("C ABI host paths: %s (%d failures)\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
