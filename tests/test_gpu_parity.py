"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative L2 over all targets and components, u and dalpha
separately): the direct P2P kernel against FP64 direct summation <= 1e-5;
the FMM at p = 10 <= 1e-4.  Lower orders are reported and must improve with p.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _vf():
    import paper_1106_5273_amd as vf
    return vf


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(case, ret_ctx=False, **kw):
    import torch
    vf = _vf()
    t = vf.case_to_device(case)
    ctx = vf.Context(**kw)
    ctx.build(t[0], t[1], t[2], t[6])
    out = ctx.evaluate(*t)
    torch.cuda.synchronize()
    u = np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64)
    da = np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64)
    if ret_ctx:
        return u, da, ctx
    ctx.close()
    return u, da


def alpha_of(case):
    return np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)


# ----------------------------------------------------------------------------
# direct P2P kernel
# ----------------------------------------------------------------------------
def _ring(n=777, seed=3):
    return wl.ring_case(n, np.random.default_rng(seed))


def _dup(n=500):
    c = wl.random_cloud(n, seed=4, L=0.3, core=0.05)
    for k in ("x", "y", "z", "ax", "ay", "az", "sigma"):
        c[k] = np.concatenate([c[k], c[k][:37]])
    c["ax"][-37:] *= 0.5
    c["n"] = n + 37
    return c


@pytest.mark.parametrize("name,make", [
    ("cloud1000", lambda: wl.random_cloud(1000, seed=1, L=1.0, core=0.05)),
    ("ring777", _ring),
    ("tg16", lambda: wl.taylor_green_case(16)),
    ("coincident", _dup),
])
@pytest.mark.parametrize("scheme", [0, 1])
def test_direct_p2p_matches_fp64(name, make, scheme):
    case = make()
    u, da = run(case, direct=1, scheme=scheme)
    ref = oracle.direct(case)
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(da))
    assert rel(u, ref["u"]) <= 1e-5
    assert rel(da, ref["da_t" if scheme == 0 else "da_c"]) <= 1e-5


def test_direct_p2p_compensated_sum():
    case = wl.random_cloud(2000, seed=9, L=1.0, core=0.05)
    u, da = run(case, direct=1, kahan=1)
    ref = oracle.direct(case)
    assert rel(u, ref["u"]) <= 1e-5 and rel(da, ref["da_t"]) <= 1e-5


# ----------------------------------------------------------------------------
# FMM, free space
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tg32_ref():
    case = wl.taylor_green_case(32)
    return case, oracle.direct(case)


def test_fmm_free_space_error_falls_with_p(tg32_ref):
    case, ref = tg32_ref
    errs = {}
    for p in (4, 6, 8, 10):
        u, da = run(case, p=p)
        errs[p] = (rel(u, ref["u"]), rel(da, ref["da_t"]))
        print("C1 taylor-green 32^3 free space p=%d: rel-L2 u %.3e dalpha %.3e" % (p, *errs[p]))
    for a, b in ((4, 6), (6, 8), (8, 10)):
        assert errs[b][0] < errs[a][0] and errs[b][1] < errs[a][1]
    assert errs[10][0] <= 1e-4 and errs[10][1] <= 1e-4


def test_fmm_classical_scheme(tg32_ref):
    case, ref = tg32_ref
    u, da = run(case, p=10, scheme=1)
    assert rel(da, ref["da_c"]) <= 1e-4


@pytest.mark.parametrize("n,ncrit", [(5000, 64), (7321, 32), (3001, 200)])
def test_fmm_adaptive_cloud(n, ncrit):
    """Clustered (adaptive, ragged leaves) input: two Gaussian blobs of particles."""
    rng = np.random.default_rng(n)
    p = np.concatenate([rng.normal(0.0, 0.15, (n // 2, 3)), rng.normal(0.6, 0.05, (n - n // 2, 3))])
    a = rng.standard_normal((n, 3)) / n
    case = dict(x=p[:, 0].astype(np.float32), y=p[:, 1].astype(np.float32), z=p[:, 2].astype(np.float32),
                ax=a[:, 0].astype(np.float32), ay=a[:, 1].astype(np.float32), az=a[:, 2].astype(np.float32),
                sigma=np.full(n, 0.01, np.float32), n=n)
    u, da = run(case, p=10, ncrit=ncrit)
    ref = oracle.direct(case)
    assert rel(u, ref["u"]) <= 1e-4 and rel(da, ref["da_t"]) <= 1e-4


def test_ring_cloud():
    case = wl.ring_case(20000, np.random.default_rng(5))
    u, da = run(case, p=8)
    idx = np.random.default_rng(0).choice(case["n"], 1500, replace=False)
    ref = oracle.direct(case, targets=idx)
    assert rel(u[idx], ref["u"]) <= 1e-4 and rel(da[idx], ref["da_t"]) <= 1e-4


# ----------------------------------------------------------------------------
# traversal coverage: every (target, source, image) particle pair exactly once
# ----------------------------------------------------------------------------
def _coverage(case, **kw):
    import torch
    vf = _vf()
    t = vf.case_to_device(case)
    with vf.Context(**kw) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        torch.cuda.synchronize()
        L = ctx.lists()
        st = ctx.stats()
    n = case["n"]
    start, count = L["cell_start"], L["cell_count"]
    nimg = st["images_traversed"] if kw.get("periodic") else 1
    ncell = start.size
    # ancestors by range containment
    leaves = np.unique(L["p2p_tgt"])
    for leaf in leaves:
        s, c = start[leaf], count[leaf]
        anc = np.nonzero((start <= s) & (start + count >= s + c))[0]
        cov = np.zeros(n * nimg, dtype=np.int64)
        sel = L["p2p_tgt"] == leaf
        for src, img in zip(L["p2p_src"][sel], L["p2p_img"][sel]):
            cov[img * n + np.arange(start[src], start[src] + count[src])] += 1
        selm = np.isin(L["m2l_tgt"], anc)
        for src, img in zip(L["m2l_src"][selm], L["m2l_img"][selm]):
            cov[img * n + np.arange(start[src], start[src] + count[src])] += 1
        assert cov.min() == 1 and cov.max() == 1, (leaf, cov.min(), cov.max())
    # every particle sits in exactly one P2P target leaf
    owned = np.zeros(n, dtype=np.int64)
    for leaf in leaves:
        owned[start[leaf]:start[leaf] + count[leaf]] += 1
    assert owned.min() == 1 and owned.max() == 1
    assert ncell == st["ncells"]


def test_traversal_coverage_free_space():
    _coverage(wl.random_cloud(3000, seed=11, L=1.0, core=0.01), p=6, ncrit=32)


def test_traversal_coverage_periodic():
    case = wl.taylor_green_case(12, periodic=True)
    _coverage(case, p=6, ncrit=16, periodic=1, box_len=2 * np.pi, images=1)


# ----------------------------------------------------------------------------
# periodic
# ----------------------------------------------------------------------------
def test_periodic_taylor_green_closed_form():
    case = wl.taylor_green_case(32, periodic=True)
    us, Js = oracle.spectral_lattice(case)
    das, _ = oracle.stretching(Js, alpha_of(case))
    u, da = run(case, p=10, periodic=1, box_len=2 * np.pi, images=5)
    assert rel(u, us) <= 1e-4 and rel(da, das) <= 1e-4


def test_periodic_turbulence_images_sweep():
    case = wl.turbulence_case(32, seed=21)
    us, Js = oracle.spectral_lattice(case)
    das, _ = oracle.stretching(Js, alpha_of(case))
    errs = {}
    for K in (1, 2, 3, 4, 6):
        u, da = run(case, p=10, periodic=1, box_len=2 * np.pi, images=K)
        errs[K] = (rel(u, us), rel(da, das))
        print("turbulence 32^3 periodic p=10 images=%d: rel-L2 u %.3e dalpha %.3e" % (K, *errs[K]))
    assert errs[6][0] <= 1e-4 and errs[6][1] <= 1e-4
    assert errs[6][0] < errs[1][0]


def test_c2_full_size_matches_spectral_oracle():
    """128^3 periodic turbulence-shaped lattice, p = 10, theta = 0.5: the
    velocity and stretching of every particle against the exact FP64 periodic
    sum, in the configuration the bench times."""
    case = wl.turbulence_case(128, seed=2)
    u, da = run(case, p=10, periodic=1, box_len=2 * np.pi, images=6)
    us, Js = oracle.spectral_lattice(case)
    das, _ = oracle.stretching(Js, alpha_of(case))
    eu, ed = rel(u, us), rel(da, das)
    print("C2 128^3: rel-L2 u %.3e dalpha %.3e" % (eu, ed))
    assert eu <= 1e-4 and ed <= 1e-4


# ----------------------------------------------------------------------------
# determinism, ordering, ABI errors
# ----------------------------------------------------------------------------
def test_bitwise_deterministic():
    import torch
    vf = _vf()
    case = wl.turbulence_case(32, seed=5)
    t = vf.case_to_device(case)
    with vf.Context(p=8, periodic=1, box_len=2 * np.pi, images=3) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        a = [o.clone() for o in ctx.evaluate(*t)]
        ctx.build(t[0], t[1], t[2], t[6])
        b = ctx.evaluate(*t)
        torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_outputs_follow_input_order():
    case = wl.random_cloud(4000, seed=13, L=1.0, core=0.02)
    perm = np.random.default_rng(1).permutation(case["n"])
    shuf = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in case.items()}
    u0, d0 = run(case, p=8)
    u1, d1 = run(shuf, p=8)
    assert rel(u1, u0[perm]) <= 1e-6 and rel(d1, d0[perm]) <= 1e-6


def test_abi_errors():
    import torch
    vf = _vf()
    case = wl.random_cloud(100, seed=2, L=1.0, core=0.05)
    t = vf.case_to_device(case)
    with vf.Context(p=6) as ctx:
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.evaluate(*t)
        ctx.build(t[0], t[1], t[2], t[6])
        with pytest.raises(vf.VfmmError, match="EINVAL"):
            ctx.evaluate(*t, out=(t[0], t[1], t[2], t[3], t[4], t[5]))
        short = tuple(x[:50].contiguous() for x in t)
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.evaluate(*short)
        bad = t[0].clone()
        bad[3] = float("nan")
        with pytest.raises(vf.VfmmError, match="EDOMAIN"):
            ctx.build(bad, t[1], t[2], t[6])
        sig = t[6].clone()
        sig[0] *= 2
        with pytest.raises(vf.VfmmError, match="EINVAL"):
            ctx.build(t[0], t[1], t[2], sig)
        e = torch.empty(0, device="cuda")
        ctx.build(e, e, e, e)
        ctx.evaluate(e, e, e, e, e, e, e)
    with vf.Context(p=6, periodic=1, box_len=0.5) as ctx:
        with pytest.raises(vf.VfmmError, match="EDOMAIN"):
            ctx.build(t[0], t[1], t[2], t[6])


# ----------------------------------------------------------------------------
# rk_step
# ----------------------------------------------------------------------------
def test_rk_step_matches_manual_heun_and_conserves_strength():
    import torch
    vf = _vf()
    case = wl.turbulence_case(16, seed=8)
    dt, nu = 0.05, 0.01
    L = 2 * np.pi
    kw = dict(p=8, periodic=1, box_len=L, images=3)
    t = [x.clone() for x in vf.case_to_device(case)]
    with vf.Context(**kw) as ctx:
        ctx.rk_step(dt, nu, *t)
        torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in t]
    # manual Heun through evaluate
    s = [x.clone() for x in vf.case_to_device(case)]
    with vf.Context(**kw) as ctx:
        ctx.build(s[0], s[1], s[2], s[6])
        k1 = ctx.evaluate(*s)
        pred = [s[i] + dt * k1[i] for i in range(3)] + [s[3 + i] + dt * k1[3 + i] for i in range(3)]
        pred = [torch.remainder(pred[i], L) if i < 3 else pred[i] for i in range(6)]
        sig2 = torch.sqrt(s[6] * s[6] + 2 * nu * dt)
        ctx.build(pred[0], pred[1], pred[2], sig2)
        k2 = ctx.evaluate(*pred, sig2)
        torch.cuda.synchronize()
    ref = [(s[i] + 0.5 * dt * (k1[i] + k2[i])).cpu().numpy() for i in range(3)]
    ref = [np.mod(r, L) for r in ref] + [(s[3 + i] + 0.5 * dt * (k1[3 + i] + k2[3 + i])).cpu().numpy() for i in range(3)]
    for i in range(6):
        assert np.abs(got[i] - ref[i]).max() <= 1e-5 * max(1.0, np.abs(ref[i]).max())
    assert np.allclose(got[6], np.sqrt(case["sigma"].astype(np.float64) ** 2 + 2 * nu * dt), rtol=1e-6)
    a0 = alpha_of(case).sum(axis=0)
    a1 = np.stack(got[3:6], 1).sum(axis=0)
    scale = np.abs(alpha_of(case)).sum()
    assert np.abs(a1 - a0).max() <= 1e-5 * scale
