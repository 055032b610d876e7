"""trevr_compute_J_noalloc (the fixed per-GPU scratch array) against
trevr_compute_J (a caller scratch tensor) on the same trees: J to the
repeat-call tolerance (sums formed with LDS atomics agree to FP32 rounding,
about 1e-7 relative; 1e-5 asserted) and every work counter equal, on two calls
in a row, the second on a smaller tree with a smaller active set, then the
first tree again; a tree whose scratch exceeds the array is refused."""
import numpy as np
import pytest

from paper_2310_15235_amd import scenes

pytestmark = pytest.mark.gpu


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_15235_amd import api
    return api


def _rel(a, b):
    floor = 1e-12 * np.abs(b).max(axis=1, keepdims=True)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), np.maximum(floor, 1e-300)))


def _pair(api, sc, act):
    import torch
    T = api.Tree.from_scene(sc)
    a = torch.as_tensor(np.ascontiguousarray(act, np.uint8), device="cuda")
    bg = None
    if sc.background:
        bg = torch.as_tensor(np.ascontiguousarray(sc.bg, np.float32), device="cuda")
    J0 = T.compute_J(a, bg).cpu().numpy()
    c0 = T.counters()
    import ctypes
    need = ctypes.c_size_t()
    api.lib().trevr_scratch_needed(T.handle, ctypes.byref(need))
    print(f"[noalloc] {sc.name}: n {sc.n}, scratch needed {need.value} bytes", flush=True)
    J1 = T.compute_J_noalloc(a, bg).cpu().numpy()
    T.check()
    c1 = T.counters()
    T.close()
    return J0, J1, c0, c1


def test_noalloc_matches_compute_J_two_calls():
    api = _api()
    big = scenes.lognormal_scene(n=12000, seed=101, grid=32, bands=(1.0, 10.0, 100.0), nside=2)
    small = scenes.isothermal_scene(n=2 ** 12, seed=102, active_frac=0.3)
    cases = [(big, big.active), (small, small.active),
             (big, scenes.active_subset(big, 0.2, 7))]
    for sc, act in cases:
        J0, J1, c0, c1 = _pair(api, sc, act)
        a = np.ones(sc.n, bool) if act is None else act.astype(bool)
        assert c0 == c1
        assert _rel(J1[:, a], J0[:, a]) < 1e-5
        assert np.all(J1[:, ~a] == 0.0)


def test_noalloc_refuses_scratch_beyond_the_array():
    api = _api()
    import torch
    sc = scenes.config_clumpy()
    T = api.Tree.from_scene(sc)
    J = torch.full((sc.n_bands, sc.n), -3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(api.TrevrError) as e:
        T.compute_J_noalloc(out=J)
    assert e.value.status == api.E_CAPACITY
    assert bool(torch.all(J == -3.0))
    import ctypes
    need = ctypes.c_size_t()
    api.lib().trevr_scratch_needed(T.handle, ctypes.byref(need))
    assert need.value > api.NOALLOC_SCRATCH_BYTES
    T.close()
