"""Velocity on a periodic probe lattice and its energy spectrum (Sec. 4.3:
the spectrum of the velocity induced on a uniform lattice of points that are
not the particles) through the C ABI, against the FP64 oracle.

* vfmm_energy_spectrum against oracle.energy_spectrum on the same velocities:
  both are float64 FFTs of the same float32 samples, so every shell agrees to
  1e-12 of the total energy.
* The periodic 128^3 turbulence-shaped particles with the 128^3 probe lattice
  at the cell corners: u at every probe against the exact zero-mean periodic
  sum at the shifted lattice (oracle.spectral_lattice with offset -h/2),
  rel-L2 <= 1e-4 and worst probe <= 1e-3 of the RMS; then E(k) of the library's
  probe velocities (computed by the library) against E(k) of the oracle's
  velocities, shell by shell: |dE(k)| <= 1e-4 E(k) + 1e-9 sum E (a velocity
  error of relative size e changes a shell's energy by about 2e of it; the
  second term covers the far tail, where E(k) falls below the error's own
  broadband energy)."""
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


@pytest.mark.parametrize("n", [16, 64])
def test_energy_spectrum_matches_oracle(n):
    import torch
    vf = _vf()
    rng = np.random.default_rng(70 + n)
    u = rng.standard_normal((n ** 3, 3)).astype(np.float32)
    u[:, 1] += np.float32(0.5)  # a mean flow puts energy into shell 0
    ref = oracle.energy_spectrum(u.astype(np.float64), n, L2PI)
    T = [torch.from_numpy(np.ascontiguousarray(u[:, k])).cuda() for k in range(3)]
    with vf.Context() as ctx:
        E = ctx.energy_spectrum(n, *T)
    print("spectrum %d^3: %d shells, max |dE| / sum E = %.2e" % (n, E.size, np.abs(E - ref).max() / ref.sum()))
    assert E.shape == ref.shape
    assert np.abs(E - ref).max() <= 1e-12 * ref.sum()
    assert abs(E.sum() - 0.5 * np.mean(np.sum(u.astype(np.float64) ** 2, 1))) <= 1e-12 * E.sum()


def test_energy_spectrum_rejects_other_sizes():
    import torch
    vf = _vf()
    x = torch.zeros(27, dtype=torch.float32, device="cuda")
    with vf.Context() as ctx:
        with pytest.raises(vf.VfmmError, match="power of two"):
            ctx.energy_spectrum(3, x, x, x)


def test_periodic_probe_lattice_full_size_and_spectrum():
    import torch
    vf = _vf()
    n = 128
    case = wl.turbulence_case(n, seed=2)
    h = case["h"]
    pts = wl.corner_lattice(n)
    us, _ = oracle.spectral_lattice(case, offset=(-0.5 * h, -0.5 * h, -0.5 * h))
    t = vf.case_to_device(case)
    T = [torch.from_numpy(p).cuda() for p in pts]
    # the periodic cube [-h/4, 2 pi - h/4)^3 puts no particle ((i + 1/2) h) and no probe (i h) on an octree face
    q = -0.25 * h
    with vf.Context(p=10, ncrit=128, periodic=1, box_len=L2PI, box_lo=(q, q, q), images=6) as ctx:
        ctx.build_targets(t[0], t[1], t[2], t[6], *T)
        out = ctx.evaluate_targets(t[3], t[4], t[5])
        st = ctx.stats()
        E = ctx.energy_spectrum(n, *out[6:9])
        torch.cuda.synchronize()
    tu = np.stack([o.cpu().numpy() for o in out[6:9]], 1).astype(np.float64)
    print("periodic probe lattice 128^3: cells %d leaves %d P2P pairs %d" % (st["ncells"], st["nleaves"],
                                                                            st["p2p_pairs"]))
    check("periodic probe lattice 128^3 u", tu, us, 1e-4, 1e-3)
    Eref = oracle.energy_spectrum(us, n, L2PI)
    dE = np.abs(E - Eref)
    bound = 1e-4 * Eref + 1e-9 * Eref.sum()
    k = np.arange(E.size)
    print("E(k), shells 1..12: library", np.array2string(E[1:13], precision=5))
    print("worst shell: k = %d, |dE| = %.3e, E = %.3e" % (k[np.argmax(dE / bound)], dE.max(), Eref[np.argmax(dE / bound)]))
    assert np.all(dE <= bound)
