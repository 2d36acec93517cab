"""rk_step and the periodic sum off the lattice against the FP64 oracle.

A Heun step (Sec. 2.1: x, alpha and sigma^2 advance together by Eqs. (1),
(3) and (4)) of the library is compared with ``oracle.heun_step`` whose two
stage rates come from the FP64 oracle: the direct sum in free space and the
exact zero-mean Fourier series in the periodic cube (the RK stage-2 particles
are off the lattice, Sec. 3.5).  The compared quantities are the increments
of one step, x1 - x0 (nearest image in the periodic cube), alpha1 - alpha0
and sigma1 - sigma0, so that the error is measured against what the step
changed, not against the unchanged state.

Tolerances: rel-L2 <= 1e-4 (the FMM gate at p = 10) for each increment and
for u, dalpha of an evaluation; the worst single target <= 1e-3 of the RMS
target magnitude (ten times the L2 gate: one target off by a tenth of the
typical magnitude fails it at any N)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import check

pytestmark = pytest.mark.gpu

L2PI = 2.0 * np.pi


def _vf():
    import paper_1106_5273_amd as vf
    return vf


def _state(case):
    x = np.stack([case["x"], case["y"], case["z"]], 1).astype(np.float64)
    a = np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)
    return x, a, np.asarray(case["sigma"], np.float64)


def _with_state(case, x, a, s):
    c = dict(case)
    c.update(x=x[:, 0], y=x[:, 1], z=x[:, 2], ax=a[:, 0], ay=a[:, 1], az=a[:, 2], sigma=s)
    return c


def _direct_rates(case):
    def rates(x, a, s):
        r = oracle.direct(_with_state(case, x, a, s))
        return r["u"], r["da_t"]
    return rates


def _series_rates(case, L, kmax):
    def rates(x, a, s):
        assert np.ptp(s) == 0.0  # the series route takes one core
        u, J = oracle.fourier_series_points(_with_state(case, x, a, s), L, kmax)
        da, _ = oracle.stretching(J, a)
        return u, da
    return rates


def _library_step(case, dt, nu, **kw):
    import torch
    vf = _vf()
    t = [x.clone() for x in vf.case_to_device(case)]
    with vf.Context(**kw) as ctx:
        ctx.rk_step(dt, nu, *t)
        torch.cuda.synchronize()
        st = ctx.stats()
    g = [x.cpu().numpy().astype(np.float64) for x in t]
    return np.stack(g[:3], 1), np.stack(g[3:6], 1), g[6], st


def _compare_step(label, case, ref, got, L=None):
    x0, a0, s0 = _state(case)
    x1, a1, s1, st = got
    dx = x1 - x0
    dxr = ref["x"] - x0
    if L is not None:
        dx = np.mod(dx + 0.5 * L, L) - 0.5 * L
        dxr = np.mod(dxr + 0.5 * L, L) - 0.5 * L
    print("%s: n=%d cells=%d leaves=%d depth=%d p2p_pairs=%d" % (label, case["n"], st["ncells"], st["nleaves"],
                                                                 st["depth"], st["p2p_pairs"]), flush=True)
    check(label + " dx", dx, dxr, 1e-4, 1e-3)
    check(label + " dalpha", a1 - a0, ref["alpha"] - a0, 1e-4, 1e-3)
    check(label + " dsigma", (s1 - s0)[:, None], (ref["sigma"] - s0)[:, None], 1e-4, 1e-3)
    if L is not None:
        lo = np.asarray(case.get("box_lo", (0.0, 0.0, 0.0)), np.float64)
        assert np.all(x1 >= lo) and np.all(x1 < lo + L), "positions left the periodic cube"


def _dt(u, h):
    """Step size of the full-step workload: a quarter spacing at the largest speed."""
    return 0.25 * h / float(np.max(np.linalg.norm(u, axis=1)))


def test_rk_step_free_space_matches_oracle_heun():
    """4,096 off-lattice particles in free space, p = 10: one library Heun
    step against the FP64 Heun step on the direct sum at both stages."""
    case = wl.jittered(wl.turbulence_case(16, seed=21), 0.4, seed=22)
    nu = 0.05
    rates = _direct_rates(case)
    dt = _dt(rates(*_state(case))[0], case["h"])
    ref = oracle.heun_step(case, dt, nu, rates)
    got = _library_step(case, dt, nu, p=10)
    _compare_step("rk_step free space 16^3 jittered", case, ref, got)
    # the transpose stretching conserves the total strength over the step
    a0 = _state(case)[1]
    assert np.abs(got[1].sum(0) - a0.sum(0)).max() <= 1e-5 * np.abs(a0).sum()


@pytest.mark.parametrize("lo", [0.0, -np.pi], ids=["cube_at_0", "cube_at_minus_pi"])
def test_rk_step_periodic_matches_oracle_heun(lo):
    """Periodic jittered 16^3 lattice, sigma = 1.5h, p = 10, leaves of 64: the
    library's Heun step against the FP64 Heun step on the exact zero-mean
    Fourier series at both stages.  In the cube [-pi, pi)^3 (whose corner is
    not a float32 number) 96 particles sit on the faces, at the float32 values
    closest to -pi and pi inside the cube, so that the step wraps some of them
    across."""
    case = wl.jittered(wl.turbulence_case(16, seed=23), 0.4, seed=24)
    if lo != 0.0:
        lo32 = np.nextafter(np.float32(lo), np.float32(0))          # smallest float32 >= lo
        hi32 = np.nextafter(np.float32(lo + L2PI), np.float32(0))   # largest float32 < lo + L
        assert float(lo32) >= lo and float(hi32) < lo + L2PI
        rng = np.random.default_rng(25)
        for k in ("x", "y", "z"):
            case[k] = np.ascontiguousarray((case[k].astype(np.float64) + lo).astype(np.float32))
            case[k] = np.where(case[k].astype(np.float64) < lo, lo32, case[k]).astype(np.float32)
            case[k] = np.where(case[k].astype(np.float64) >= lo + L2PI, hi32, case[k]).astype(np.float32)
        face = rng.choice(case["n"], 96, replace=False)
        for j, i in enumerate(face):
            k = ("x", "y", "z")[j % 3]
            case[k][i] = lo32 if j % 2 == 0 else hi32
        case["box_lo"] = (lo, lo, lo)
    nu = 0.05
    rates = _series_rates(case, L2PI, 16)
    dt = _dt(rates(*_state(case))[0], case["h"])
    ref = oracle.heun_step(case, dt, nu, rates, L=L2PI, lo=(lo, lo, lo))
    got = _library_step(case, dt, nu, p=10, periodic=1, box_lo=(lo, lo, lo), box_len=L2PI, images=6)
    _compare_step("rk_step periodic 16^3 jittered lo=%.4f" % lo, case, ref, got, L=L2PI)


def test_periodic_jittered_lattice_matches_fourier_series():
    """32^3 turbulence-shaped field moved off the lattice (each coordinate by
    up to 0.75 h, so particles leave their lattice cells), sigma = 1.5h,
    p = 10, leaves of <= 64 particles: velocity and stretching of every
    particle against the exact zero-mean Fourier series (the particles stage 2
    of an RK step sees).  Leaves then hold unequal counts, overfull ones split
    a level deeper, and the near field meets all three cutoff forms."""
    import torch
    vf = _vf()
    case = wl.jittered(wl.turbulence_case(32, seed=26), 0.75, seed=27)
    us, Js = oracle.fourier_series_points(case, L2PI, 30)
    das, _ = oracle.stretching(Js, _state(case)[1])
    t = vf.case_to_device(case)
    with vf.Context(p=10, ncrit=64, periodic=1, box_len=L2PI, images=6) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        out = ctx.evaluate(*t)
        torch.cuda.synchronize()
        st = ctx.stats()
    u = np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64)
    da = np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64)
    print("jittered 32^3: cells=%d leaves=%d depth=%d p2p_pairs=%d m2l=%d" % (
        st["ncells"], st["nleaves"], st["depth"], st["p2p_pairs"], st["m2l_entries"]), flush=True)
    assert st["depth"] >= 4  # some leaves overflowed 64 and split
    check("jittered 32^3 u", u, us, 1e-4, 1e-3)
    check("jittered 32^3 dalpha", da, das, 1e-4, 1e-3)
