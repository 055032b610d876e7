"""Adjoint (compute_J_backward) versus the oracle's forward-mode derivative.

The oracle differentiates its FP64 algorithm with dual numbers, every
discrete decision frozen at its value.  For E = <gJ, J> the adjoint gives
dE/d(L, kappa, rho); the oracle gives the directional derivative
dE/dt = <gJ, dJ/dt> for any direction t, so

  * dot-product tests: <g_gpu, t> = <gJ, JVP_oracle(t)> for random t;
  * sampled components: t = a unit vector gives one gradient component.

Tolerances: the adjoint's per-term arithmetic is FP32 like the forward's
(relative error ~1e-6 per term, summed in FP64), and gradient components
are sums of terms of both signs (h enters the intensity kernel, the p-p
columns, the bucket absorption and the thick factor), so a component is
checked to 1e-4 of its value plus 1e-6 of the largest component of its
array, and a dot product to 1e-4 of the sum of the magnitudes of its
terms.
"""
import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes

pytestmark = pytest.mark.gpu


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_15235_amd import api
    return api


def _close(got, ref, rtol):
    """|got - ref| <= rtol |ref| + 1e-6 max|ref|: gradient sums are formed
    with atomics (FP32 in LDS, FP64 in memory), so repeated runs agree to
    FP32 rounding of the partial sums, and components that cancel keep an
    absolute error on the scale of the array's largest entries."""
    tol = rtol * np.abs(ref) + 1e-6 * np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= tol), float(np.max(np.abs(got - ref) - tol))


def _weights(sc, active, seed):
    rng = np.random.default_rng(seed)
    gJ = rng.normal(size=(sc.n_bands, sc.n))
    gJ[:, ~active.astype(bool)] = 0.0
    return gJ


def _dot_check(sc, active, seed=0, ndir=3, extra_flags=0):
    api = _api()
    act = np.ones(sc.n, np.uint8) if active is None else active
    gJ = _weights(sc, act, seed)
    gL, gk, gr = api.compute_J_backward(sc, gJ, active=act, extra_flags=extra_flags)
    assert np.all(np.isfinite(gL)) and np.all(np.isfinite(gk)) and np.all(np.isfinite(gr))
    rng = np.random.default_rng(seed + 100)
    B, n = sc.n_bands, sc.n
    for d in range(ndir):
        which = d % 3
        tL = rng.normal(size=(B, n)) * sc.lum if which == 0 else None
        tk = rng.normal(size=(B, n)) * sc.kappa if which == 1 else None
        tr = rng.normal(size=n) * sc.rho if which == 2 else None
        _, dJ, _ = oracle.jvp(sc, tL=tL, tkappa=tk, trho=tr, active=act)
        lhs = float(np.sum(gJ * dJ))
        terms = [g * t for g, t in ((gL, tL), (gk, tk), (gr, tr)) if t is not None]
        rhs = float(sum(np.sum(x) for x in terms))
        scale = max(float(np.sum(np.abs(gJ * dJ))), float(sum(np.sum(np.abs(x)) for x in terms)))
        assert scale > 0
        assert abs(lhs - rhs) <= 1e-4 * scale, (["L", "kappa", "rho"][which], lhs, rhs, scale)
    return gL, gk, gr, gJ


def _component_check(sc, active, gJ, grads, picks_per_array=4, seed=1):
    """Sampled components: the largest and some random ones of each array."""
    rng = np.random.default_rng(seed)
    names = ("L", "kappa", "rho")
    for name, g in zip(names, grads):
        flat = np.abs(g).ravel()
        idx = list(np.argsort(flat)[-2:]) + list(rng.choice(flat.size, picks_per_array - 2,
                                                             replace=False))
        gmax = flat.max()
        for fi in idx:
            t = np.zeros(g.size)
            t[fi] = 1.0
            t = t.reshape(g.shape)
            kw = {"L": dict(tL=t), "kappa": dict(tkappa=t), "rho": dict(trho=t)}[name]
            _, dJ, _ = oracle.jvp(sc, active=active, **kw)
            go = float(np.sum(gJ * dJ))
            gg = float(g.ravel()[fi])
            assert abs(gg - go) <= 1e-4 * abs(go) + 1e-6 * gmax, (name, int(fi), gg, go, gmax)


SCENES = {
    "tiny_lognormal_nside1": lambda: scenes.lognormal_scene(n=3000, seed=51, grid=16,
                                                            bands=(1.0, 10.0), nside=1),
    "lognormal_nside2_3bands": lambda: scenes.lognormal_scene(n=6000, seed=52, grid=16,
                                                              bands=(1.0, 10.0, 100.0), nside=2),
    "uniform_nside4": lambda: scenes.uniform_scene(n=3000, seed=53, n_src=60, bands=(1.0, 4.0),
                                                   nside=4),
    "no_near_field": lambda: scenes.uniform_scene(n=3000, seed=54, n_src=80, bands=(2.0,),
                                                  nside=2, near_field=False),
    "no_thick": lambda: scenes.lognormal_scene(n=3000, seed=55, grid=16, bands=(1.0, 10.0),
                                               nside=2, thick_corr=False),
    "background": lambda: scenes.isothermal_scene(n=4000, seed=56, active_frac=1.0),
    "leaf12_many_bands": lambda: scenes.lognormal_scene(n=3000, seed=57, grid=16,
                                                        bands=(0.5, 1, 2, 4, 8), nside=2,
                                                        leaf_size=12),
    "rpp_min": lambda: scenes.uniform_scene(n=2000, seed=58, n_src=40, bands=(1.0,), nside=2,
                                            rpp_min=0.1),
    "eight_bands": lambda: scenes.lognormal_scene(n=3000, seed=60, grid=16,
                                                  bands=tuple(float(2 ** k) for k in range(8)),
                                                  nside=2),
    "ten_bands": lambda: scenes.lognormal_scene(n=3000, seed=63, grid=16,
                                                bands=tuple(float(2 ** (k / 2)) for k in range(10)),
                                                nside=2),
    "absorption_average": lambda: scenes.lognormal_scene(n=4000, seed=64, grid=16,
                                                         bands=(1.0, 10.0), nside=2,
                                                         absorption_avg=True),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_adjoint_dot_products(name):
    sc = SCENES[name]()
    _dot_check(sc, sc.active)


@pytest.mark.parametrize("name", ["tiny_lognormal_nside1", "lognormal_nside2_3bands",
                                  "background"])
def test_adjoint_sampled_components(name):
    sc = SCENES[name]()
    act = np.ones(sc.n, np.uint8) if sc.active is None else sc.active
    gL, gk, gr, gJ = _dot_check(sc, act, ndir=0)
    _component_check(sc, act, gJ, (gL, gk, gr))


def test_adjoint_ragged_active_subset():
    sc = scenes.lognormal_scene(n=8000, seed=59, grid=16, bands=(1.0, 10.0), nside=2)
    act = scenes.active_subset(sc, 0.02, 3)
    gL, gk, gr, gJ = _dot_check(sc, act)
    _component_check(sc, act, gJ, (gL, gk, gr), picks_per_array=3, seed=2)


@pytest.mark.parametrize("keep", [False, True], ids=["recompute", "keep_depths"])
def test_adjoint_differentiation_full_size_dot(keep):
    """2^18 elements, 2 bands, N_side 2 at full size; the objective weights
    1% of the receivers so the oracle's derivative finishes in seconds.  The
    adjoint recomputes the rays' optical-depth prefixes, or (KEEP_DEPTHS)
    reads the depths the forward kept."""
    api = _api()
    sc = scenes.config_differentiation()
    act = scenes.active_subset(sc, 0.01, 7)
    _dot_check(sc, act, seed=7, ndir=8, extra_flags=api.KEEP_DEPTHS if keep else 0)


@pytest.mark.parametrize("name", ["lognormal_nside2_3bands", "uniform_nside4", "background"])
def test_adjoint_keep_depths_matches_recompute(name):
    """The kept far-source depths are the forward's own, so the adjoint with
    KEEP_DEPTHS equals the recomputing one up to FP32 rounding of sums formed
    with atomics."""
    api = _api()
    sc = SCENES[name]()
    act = np.ones(sc.n, np.uint8) if sc.active is None else sc.active
    gJ = _weights(sc, act, 3)
    a = api.compute_J_backward(sc, gJ, active=act)
    b = api.compute_J_backward(sc, gJ, active=act, extra_flags=api.KEEP_DEPTHS)
    for x, y in zip(a, b):
        tol = 1e-5 * np.abs(x) + 1e-7 * np.abs(x).max()
        assert np.all(np.abs(x - y) <= tol), float(np.max(np.abs(x - y) - tol))


def test_autograd_matches_abi():
    api = _api()
    import torch
    sc = scenes.lognormal_scene(n=3000, seed=60, grid=16, bands=(1.0, 10.0), nside=2)
    dev = torch.device("cuda")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    x, y, z, m = f(sc.x), f(sc.y), f(sc.z), f(sc.m)
    rho = f(sc.rho).requires_grad_(True)
    kappa = f(sc.kappa).requires_grad_(True)
    lum = f(sc.lum).requires_grad_(True)
    opts = dict(nside=sc.nside, leaf_size=sc.leaf_size, theta=sc.theta,
                flags=api.THICK_CORR | api.NEAR_FIELD, box=sc.box)
    J = api.TrevrJ.apply(x, y, z, m, rho, kappa, lum, None, None, opts)
    w = torch.as_tensor(np.random.default_rng(4).normal(size=J.shape), device=dev)
    (w * J).sum().backward()
    gL, gk, gr = api.compute_J_backward(sc, w.cpu().numpy())
    for got, ref in ((lum.grad, gL), (kappa.grad, gk), (rho.grad, gr)):
        _close(got.cpu().numpy().astype(np.float64), ref, 1e-5)
    Jo, _ = oracle.compute_J(sc)
    assert np.max(np.abs(J.detach().cpu().numpy() - Jo) / np.maximum(np.abs(Jo), 1e-300)) < 1e-4


def test_adjoint_repeatable_and_tree_unchanged():
    """A backward call leaves the tree, the forward result (to FP32 rounding of
    the atomic optical-depth sums) and the work counters unchanged."""
    api = _api()
    import torch
    sc = scenes.lognormal_scene(n=3000, seed=61, grid=16, bands=(1.0,), nside=1)
    T = api.Tree.from_scene(sc)
    J1 = T.compute_J().cpu().numpy()
    c1 = T.counters()
    g = torch.ones((1, sc.n), dtype=torch.float64, device="cuda")
    a = [x.cpu().numpy() for x in T.compute_J_backward(g)]
    b = [x.cpu().numpy() for x in T.compute_J_backward(g)]
    for u, v in zip(a, b):
        _close(u, v, 1e-5)
    J2 = T.compute_J().cpu().numpy()
    T.check()
    assert T.counters() == c1
    _close(J2, J1, 1e-6)
    T.close()


def test_adjoint_reuses_forward_state_only_for_the_same_active_set():
    """A backward after compute_J on the same scratch takes the forward's
    setup; one after the active array changed in place recomputes it.  Both
    must equal a backward on a fresh tree."""
    api = _api()
    import torch
    sc = scenes.lognormal_scene(n=4000, seed=62, grid=16, bands=(1.0, 10.0), nside=2)
    a1 = torch.as_tensor(scenes.active_subset(sc, 0.5, 1), device="cuda")
    a2 = scenes.active_subset(sc, 0.3, 2)
    g = torch.as_tensor(np.random.default_rng(9).normal(size=(2, sc.n)), device="cuda")
    T = api.Tree.from_scene(sc)
    T.compute_J(a1)
    T.compute_J(a1)                      # the scratch now fits; state recorded
    reused = [x.cpu().numpy() for x in T.compute_J_backward(g, a1)]
    a1.copy_(torch.as_tensor(a2, device="cuda"))   # same pointer, new contents
    redone = [x.cpu().numpy() for x in T.compute_J_backward(g, a1)]
    T.check()
    T.close()
    for act, got in ((scenes.active_subset(sc, 0.5, 1), reused), (a2, redone)):
        F = api.Tree.from_scene(sc)
        ref = [x.cpu().numpy() for x in
               F.compute_J_backward(g, torch.as_tensor(act, device="cuda"))]
        F.close()
        for u, v in zip(got, ref):
            _close(u, v, 1e-5)


def test_adjoint_with_scratch_shared_between_trees():
    """Tree B's forward on a scratch shared with tree A overwrites A's state;
    A's backward must then recompute, not reuse B's setup."""
    api = _api()
    import torch
    sa = scenes.lognormal_scene(n=3000, seed=63, grid=16, bands=(1.0, 10.0), nside=2)
    sb = scenes.uniform_scene(n=2000, seed=64, n_src=50, bands=(1.0, 10.0), nside=2)
    g = torch.as_tensor(np.random.default_rng(10).normal(size=(2, sa.n)), device="cuda")
    A = api.Tree.from_scene(sa)
    A.compute_J()
    A.compute_J_backward(g)              # sizes A's scratch for the backward
    Bt = api.Tree.from_scene(sb)
    Bt._scratch = A.scratch              # share it
    Bt.compute_J()
    assert Bt.scratch.data_ptr() == A.scratch.data_ptr()   # it fitted: B wrote A's scratch
    got = [x.cpu().numpy() for x in A.compute_J_backward(g)]
    A.check()
    Bt.check()
    F = api.Tree.from_scene(sa)
    ref = [x.cpu().numpy() for x in F.compute_J_backward(g)]
    for u, v in zip(got, ref):
        _close(u, v, 1e-5)
    for t in (A, Bt, F):
        t.close()


def test_adjoint_with_large_stack_and_short_cut_lists():
    """The adjoint on a tree tuned to fall back to the large traversal stack
    and to re-walk with longer cut lists, or to find most p-p sets again in
    the list fill, equals the default one."""
    api = _api()
    import torch
    sc = scenes.lognormal_scene(n=5000, seed=65, grid=16, bands=(1.0, 10.0), nside=2)
    g = torch.as_tensor(np.random.default_rng(11).normal(size=(2, sc.n)), device="cuda")
    out = []
    for tune in ((), ((api.TUNE_STACK, 64), (api.TUNE_CUT, 64)), ((api.TUNE_STAGE, 64),)):
        T = api.Tree.from_scene(sc)
        for k, v in tune:
            T.tune(k, v)
        T.compute_J()
        out.append([x.cpu().numpy() for x in T.compute_J_backward(g)])
        T.check()
        T.close()
    for tuned in out[1:]:
        for u, v in zip(out[0], tuned):
            _close(u, v, 1e-5)


@pytest.mark.parametrize("which", ["kappa", "rho", "lum"])
def test_adjoint_against_central_differences_on_the_small_copy(which):
    """The differentiation workload's 2^12-element copy (2 bands, N_side 2):
    the GPU adjoint of E = <w, J> against FP64 central differences of the
    oracle with relative step 1e-6 along x (1 + h v), the counted discrete
    decisions unmoved within the step.  J components at a kink of the map --
    a column profile where an impact parameter meets an element's size, or a
    maximum with a tie (the p-p radius rule max h/w: elements of one grid
    cell of the log-normal medium share rho and m, hence h), where the
    frozen-decision derivative takes the first tied element's slope and a
    central difference their mean -- have different one-sided quotients;
    they are skipped (weight zero) and counted."""
    api = _api()
    sc = scenes.config_differentiation_small()
    act = np.ones(sc.n, np.uint8)
    rng = np.random.default_rng({"kappa": 11, "rho": 12, "lum": 13}[which])
    w = rng.normal(size=(sc.n_bands, sc.n))
    base = dict(lum=sc.lum.astype(np.float64), kappa=sc.kappa.astype(np.float64),
                rho=sc.rho.astype(np.float64))
    v = rng.normal(size=base[which].shape)
    eps = 1e-6
    Js, cnt = [], []
    for sgn in (+1, 0, -1):
        kw = dict(base)
        kw[which] = base[which] * (1.0 + sgn * eps * v)
        J, _, c = oracle.jvp(sc, active=act, **kw)
        Js.append(J)
        cnt.append(c)
    strip = lambda c: {k: v for k, v in c.items() if k != "near_src_hits"}
    assert strip(cnt[0]) == strip(cnt[1]) == strip(cnt[2]), \
        "a counted decision moved within the step"
    right, left = (Js[0] - Js[1]) / eps, (Js[1] - Js[2]) / eps
    central = (Js[0] - Js[2]) / (2 * eps)
    den = np.maximum(np.abs(central), 1e-3 * np.abs(central).max(axis=1, keepdims=True))
    kink = np.abs(right - left) / den > 1e-4
    # observed: 12.5% of J components for rho directions (ties of the p-p
    # radius maximum), none for kappa and L
    assert kink.mean() <= (0.15 if which == "rho" else 0.0), kink.mean()
    w[kink] = 0.0
    gL, gk, gr = api.compute_J_backward(sc, w, active=act)
    g = {"lum": gL, "kappa": gk, "rho": gr}[which]
    terms = g * base[which] * v
    lhs = float(np.sum(terms))
    rhs = float(np.sum(w * central))
    scale = max(float(np.sum(np.abs(terms))), float(np.sum(np.abs(w * central))))
    print(f"{which}: {int(kink.sum())} of {kink.size} components at a kink skipped")
    assert abs(lhs - rhs) <= 1e-4 * scale, (lhs, rhs, scale, int(kink.sum()))


def test_adjoint_directed_rays():
    """The adjoint with directed rays (the source-position adjoint uses the
    aimed direction of the ray its source sits on)."""
    sc = scenes.lognormal_scene(n=4000, seed=65, grid=16, bands=(1.0, 10.0), nside=2,
                                directed=(0.31, 0.62, 0.45))
    _dot_check(sc, sc.active)


def test_adjoint_against_central_differences_tie_free_copy():
    """The 2^12 copy with every element's mass jittered by up to 1% (so no
    two elements of a grid cell share their size h and the p-p radius
    maximum has no ties): central differences along rho leave almost no
    component at a kink, and the adjoint matches them."""
    api = _api()
    sc = scenes.config_differentiation_small()
    rng = np.random.default_rng(21)
    sc = sc.with_(m=(sc.m * (1.0 + 0.01 * rng.random(sc.n))).astype(np.float32))
    act = np.ones(sc.n, np.uint8)
    w = rng.normal(size=(sc.n_bands, sc.n))
    base = sc.rho.astype(np.float64)
    v = rng.normal(size=sc.n)
    eps = 1e-6
    Js = [oracle.jvp(sc, active=act, rho=base * (1.0 + sgn * eps * v))[0] for sgn in (+1, 0, -1)]
    right, left = (Js[0] - Js[1]) / eps, (Js[1] - Js[2]) / eps
    central = (Js[0] - Js[2]) / (2 * eps)
    den = np.maximum(np.abs(central), 1e-3 * np.abs(central).max(axis=1, keepdims=True))
    kink = np.abs(right - left) / den > 1e-4
    print(f"tie-free rho: {int(kink.sum())} of {kink.size} components at a kink skipped")
    assert kink.mean() < 0.005, kink.mean()
    w[kink] = 0.0
    _, _, gr = api.compute_J_backward(sc, w, active=act)
    terms = gr * base * v
    lhs, rhs = float(np.sum(terms)), float(np.sum(w * central))
    scale = max(float(np.sum(np.abs(terms))), float(np.sum(np.abs(w * central))))
    assert abs(lhs - rhs) <= 1e-4 * scale, (lhs, rhs, scale)


def test_adjoint_per_component_small_copy():
    """64 components of each gradient array of the 2^12 copy -- the 16
    largest, the 16 smallest nonzero and 32 random -- each against the
    oracle's forward-mode derivative along that component's unit vector:
    |g - g_oracle| <= 1e-4 |g_oracle| + 1e-7 max|g| (per-term FP32
    arithmetic; a component that is a sum of terms of both signs keeps an
    absolute error on the scale of its largest terms)."""
    api = _api()
    sc = scenes.config_differentiation_small()
    act = np.ones(sc.n, np.uint8)
    rng = np.random.default_rng(31)
    gJ = rng.normal(size=(sc.n_bands, sc.n))
    grads = api.compute_J_backward(sc, gJ, active=act)
    worst = {}
    for name, g in zip(("L", "kappa", "rho"), grads):
        flat = np.abs(g).ravel()
        order = np.argsort(flat)
        nz = order[flat[order] > 0]
        picks = list(nz[-16:]) + list(nz[:16]) + list(rng.choice(flat.size, 32, replace=False))
        gmax = flat.max()
        errs = []
        for fi in picks:
            t = np.zeros(g.size)
            t[fi] = 1.0
            t = t.reshape(g.shape)
            kw = {"L": dict(tL=t), "kappa": dict(tkappa=t), "rho": dict(trho=t)}[name]
            _, dJ, _ = oracle.jvp(sc, active=act, **kw)
            go = float(np.sum(gJ * dJ))
            gg = float(g.ravel()[fi])
            errs.append(abs(gg - go) / (abs(go) + 1e-12 * gmax))
            assert abs(gg - go) <= 1e-4 * abs(go) + 1e-7 * gmax, (name, int(fi), gg, go, gmax)
        worst[name] = max(errs)
    print("largest relative component errors:", worst)
