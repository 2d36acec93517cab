"""fmm_direct_static, the entry point that allocates no device memory, against
the existing direct-mode path (fmm_build + fmm_evaluate with direct = 1) whose
kernels it shares, and against the FP64 direct sum (Eqs. 1-3) at the direct
P2P bar (rel-L2 <= 1e-5): two calls in a row on one context, the second with a
smaller input, each bitwise equal to the existing path's outputs."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _vf():
    import paper_1106_5273_amd as vf
    return vf


def _host(out):
    return (np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64),
            np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64))


def _existing(case, **kw):
    import torch
    vf = _vf()
    t = vf.case_to_device(case)
    with vf.Context(direct=1, **kw) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        out = ctx.evaluate(*t)
        torch.cuda.synchronize()
    return _host(out)


def _varcores(case, seed):
    c = dict(case)
    c["sigma"] = (case["sigma"].astype(np.float64) * np.random.default_rng(seed).uniform(0.6, 1.6, case["n"])
                  ).astype(np.float32)
    return c


@pytest.mark.parametrize("kw", [dict(), dict(scheme=1, precision=1)], ids=["transpose_float32", "classical_mixed"])
def test_static_entry_point_matches_existing_direct_path(kw):
    import torch
    vf = _vf()
    first = wl.random_cloud(60000, seed=51, L=1.0, core=0.01)
    second = _varcores(wl.random_cloud(1500, seed=52, L=0.4, core=0.02), 53)
    key = "da_t" if kw.get("scheme", 0) == 0 else "da_c"
    with vf.Context(**kw) as ctx:
        # the first launch of a kernel in a process loads its code object into
        # device memory (the HIP runtime's, not the library's): warm up first
        ctx.direct_static(*vf.case_to_device(wl.random_cloud(300, seed=50, L=1.0, core=0.05)))
        torch.cuda.synchronize()
        for k, case in enumerate((first, second)):
            t = vf.case_to_device(case)
            out = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            ctx.direct_static(*t, out=out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            u, da = _host(out)
            ru, rda = _existing(case, **kw)
            sub = np.arange(0, case["n"], max(1, case["n"] // 700))
            ref = oracle.direct(case, targets=sub)
            eu = float(np.linalg.norm(u[sub] - ref["u"]) / np.linalg.norm(ref["u"]))
            ed = float(np.linalg.norm(da[sub] - ref[key]) / np.linalg.norm(ref[key]))
            print("call %d: n=%d rel-L2 vs FP64 u %.2e dalpha %.2e, bitwise equal to direct mode: %s, "
                  "device free memory change %d bytes" % (k, case["n"], eu, ed,
                                                          np.array_equal(u, ru) and np.array_equal(da, rda),
                                                          free0 - free1), flush=True)
            assert np.array_equal(u, ru) and np.array_equal(da, rda)
            assert eu <= 1e-5 and ed <= 1e-5
            assert abs(free0 - free1) < (2 << 20)  # no device allocation (the scratch is 6.7 MB)


def test_static_entry_point_limits_and_errors():
    import torch
    vf = _vf()
    case = wl.random_cloud(100, seed=54, L=1.0, core=0.05)
    t = vf.case_to_device(case)
    with vf.Context() as ctx:
        big = torch.zeros(vf.STATIC_MAX_N + 1, dtype=torch.float32, device="cuda")
        with pytest.raises(vf.VfmmError, match="EINVAL.*VFMM_STATIC_MAX_N"):
            ctx.direct_static(*([big] * 7))
        with pytest.raises(vf.VfmmError, match="EINVAL"):
            ctx.direct_static(*t, out=(t[0], t[1], t[2], t[3], t[4], t[5]))
        sig = t[6].clone()
        sig[3] = 0.0
        with pytest.raises(vf.VfmmError, match="EDOMAIN"):
            ctx.direct_static(t[0], t[1], t[2], t[3], t[4], t[5], sig)
        e = torch.empty(0, device="cuda")
        ctx.direct_static(e, e, e, e, e, e, e)
        u, da = _host(ctx.direct_static(*t))  # still usable after the errors
        ref = oracle.direct(case)
        assert np.linalg.norm(u - ref["u"]) <= 1e-5 * np.linalg.norm(ref["u"])
    with vf.Context(periodic=1, box_len=1.0) as ctx:
        with pytest.raises(vf.VfmmError, match="free space only"):
            ctx.direct_static(*t)
    with vf.Context(precision=2) as ctx:
        with pytest.raises(vf.VfmmError, match="float32 and mixed"):
            ctx.direct_static(*t)
