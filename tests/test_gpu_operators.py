"""The far-field operators one at a time (Sec. 3.1: P2M, M2M, L2L, L2P)
through vfmm_copy_expansions, against their definitions in the FP64
expansion oracle (oracle/expansions.py, pinned in
test_oracle_pins_expansions.py).  Two Gaussian clusters give a deep,
adaptive tree (p = 8, leaves of <= 32 particles).

* P2M: each leaf's coefficients against Mt_n^m = sum_j q_j conj(R_n^m((x_j - c)/s))
  over its particles.
* M2M exactness: each internal cell's coefficients against the same sum over
  every particle below it.  Translating a degree-p multipole to the parent
  loses nothing at degree <= p, so only rounding separates the two.
* L2L exactness: a cell that receives no translation of its own holds its
  parent's local polynomial re-expanded, so both evaluate to the same
  potential at points in the cell (a tree of two tiny clusters in opposite
  corners, whose chains of single-child cells receive none).
* L2P: the far-field u and dalpha at every particle against the curl and the
  gradient (fourth-order differences of the FP64 polynomial) of its leaf's
  local expansion, contracted with alpha_i as Eq. (3) reads.
* M2L: with the strengths of one of the two corner clusters set to zero, its
  particles' velocity is the other cluster's field carried P2M -> M2M -> one
  M2L -> L2L -> L2P; in the float64 form its error against the FP64 direct sum
  falls geometrically with p (by the ratio of the expansion radii to the
  centres' distance) down to float64 rounding.
Bounds: float64 form near float64 rounding (the translations run in float64);
float32 and mixed forms from float32 storage and arithmetic.  A dropped term,
a wrong sign or a transposed index changes some coefficient by its own size,
far above every bound."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import expansions as ex

pytestmark = pytest.mark.gpu

P = 8
# (coefficient error / largest coefficient of the cell, potential, far field)
BOUNDS = {2: (1e-12, 1e-11, 1e-7), 1: (3e-5, 2e-5, 1e-4), 0: (3e-5, 2e-5, 1e-4)}


def _vf():
    import paper_1106_5273_amd as vf
    return vf


def _evaluate(case, prec, **kw):
    vf = _vf()
    import torch
    t = vf.case_to_device(case)
    with vf.Context(p=P, ncrit=32, precision=prec, **kw) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t)
        torch.cuda.synchronize()
        E = ctx.expansions()
        Ls = ctx.lists()
        st = ctx.stats()
    perm = Ls["perm"]
    pos = np.stack([case["x"], case["y"], case["z"]], 1).astype(np.float64)[perm]
    alpha = np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)[perm]
    print("\nform %d: %d cells, depth %d, %d leaves, %d M2L entries" % (prec, st["ncells"], st["depth"],
                                                                       st["nleaves"], st["m2l_entries"]))
    return dict(prec=prec, E=E, L=Ls, pos=pos, alpha=alpha, q=ex.strengths(alpha), st=st)


@pytest.fixture(scope="module", params=[2, 0, 1], ids=["float64", "float32", "mixed"])
def tree(request):
    return _evaluate(wl.clustered_cloud(3000, seed=81), request.param)


@pytest.fixture(scope="module", params=[2, 0, 1], ids=["float64", "float32", "mixed"])
def chain_tree(request):
    """Two tiny clusters in opposite corners of the fixed root cube [0, 1)^3:
    each hangs below a chain of single-child cells, the clusters meet by M2L
    near the top, and the chain cells below receive no translation of their own."""
    case = wl.clustered_cloud(600, seed=83, centres=((0.1, 0.1, 0.1), (0.9, 0.9, 0.9)), width=0.004, core=0.0004)
    return _evaluate(case, request.param, box_lo=(0.0, 0.0, 0.0), box_len=1.0)


def _cell_of_particles(n, start, count, cells):
    """For each of the n particles (sorted order), the cell among `cells` that holds it."""
    owner = np.full(n, -1)
    for c in cells:
        owner[start[c]:start[c] + count[c]] = c
    return owner


def _check_multipoles(tr, cells, what):
    E, Ls = tr["E"], tr["L"]
    geo = E["geo"]
    start, count = Ls["cell_start"], Ls["cell_count"]
    bound = BOUNDS[tr["prec"]][0]
    worst = 0.0
    # group the particles of each cell (cells of one level hold disjoint particle ranges)
    levels = sorted(set(E["level"][cells]))
    for lv in levels:
        cs = [c for c in cells if E["level"][c] == lv]
        grp = np.concatenate([np.full(count[c], i) for i, c in enumerate(cs)])
        idx = np.concatenate([np.arange(start[c], start[c] + count[c]) for c in cs])
        cen = geo[cs, :3][grp]
        side = geo[cs, 3][grp]
        ref = ex.multipoles(tr["pos"][idx], tr["q"][idx], cen, side, grp, len(cs), P)
        ref = ex.compact_from_full(ref, P)
        got = E["mult"][cs]
        err = np.abs(got - ref).max(axis=(1, 2)) / np.abs(ref).max(axis=(1, 2))
        worst = max(worst, float(err.max()))
    print("%s, form %d: %d cells, worst coefficient error %.2e of the cell's largest (bound %.0e)" %
          (what, tr["prec"], len(cells), worst, bound))
    assert worst <= bound


def test_p2m_matches_the_definition(tree):
    leaves = np.nonzero(tree["E"]["nchild"] == 0)[0]
    _check_multipoles(tree, list(leaves), "P2M")


def test_m2m_is_exact(tree):
    internal = np.nonzero(tree["E"]["nchild"] > 0)[0]
    assert internal.size >= 20 and tree["st"]["depth"] >= 5
    _check_multipoles(tree, list(internal), "M2M")


def test_l2l_is_exact_where_a_cell_has_no_translation_of_its_own(chain_tree):
    tree = chain_tree
    E, Ls = tree["E"], tree["L"]
    geo = E["geo"]
    own = np.bincount(Ls["m2l_tgt"], minlength=geo.shape[0])
    loc = ex.full_from_compact(E["loc"], P)
    cells = [c for c in range(geo.shape[0]) if own[c] == 0 and E["parent"][c] >= 0
             and np.abs(loc[E["parent"][c]]).max() > 0]
    assert len(cells) >= 3, len(cells)
    rng = np.random.default_rng(7)
    k = 8
    cs = np.repeat(cells, k)
    par = E["parent"][cs]
    x = geo[cs, :3] + 0.5 * geo[cs, 3][:, None] * rng.uniform(-1, 1, (cs.size, 3))
    psi_c = ex.potential_local(loc[cs], geo[cs, :3], geo[cs, 3], x, P)
    psi_p = ex.potential_local(loc[par], geo[par, :3], geo[par, 3], x, P)
    err = np.abs(psi_c - psi_p).max() / np.abs(psi_p).max()
    bound = BOUNDS[tree["prec"]][1]
    print("L2L, form %d: %d cells without own translations, potential error %.2e of the largest (bound %.0e)" %
          (tree["prec"], len(cells), err, bound))
    assert err <= bound


def test_l2p_matches_the_derivatives_of_the_local_expansion(tree):
    E, Ls = tree["E"], tree["L"]
    geo = E["geo"]
    leaves = np.nonzero(E["nchild"] == 0)[0]
    owner = _cell_of_particles(tree["pos"].shape[0], Ls["cell_start"], Ls["cell_count"], leaves)
    assert (owner >= 0).all()
    loc = ex.full_from_compact(E["loc"], P)
    u, J = ex.velocity_local(loc[owner], geo[owner, :3], geo[owner, 3], tree["pos"], P)
    da_t, _ = oracle.stretching(J, tree["alpha"])  # the library's default (transpose) reading of Eq. (3)
    bound = BOUNDS[tree["prec"]][2]
    for name, got, ref in (("u", E["far_u"].T, u), ("dalpha", E["far_da"].T, da_t)):
        rms = np.sqrt(np.mean(np.sum(ref * ref, 1)))
        err = np.abs(got - ref).max() / rms
        print("L2P %s, form %d: worst particle %.2e of the rms (bound %.0e)" % (name, tree["prec"], err, bound))
        assert err <= bound


def test_copy_expansions_needs_an_evaluation():
    vf = _vf()
    case = wl.clustered_cloud(500, seed=82)
    t = vf.case_to_device(case)
    with vf.Context(p=6, ncrit=32) as ctx:
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.expansions()
        ctx.build(t[0], t[1], t[2], t[6])
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.expansions()
        ctx.evaluate(*t)
        E = ctx.expansions()
        assert E["mult"].shape[1:] == (3, 28)
        ctx.build(t[0], t[1], t[2], t[6])  # a new build invalidates the expansions
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.expansions()
    with vf.Context(direct=1) as ctx:
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t)
        with pytest.raises(vf.VfmmError, match="ESTATE"):
            ctx.expansions()


def test_m2l_chain_error_falls_geometrically_with_p():
    vf = _vf()
    import torch
    case = wl.clustered_cloud(600, seed=83, centres=((0.1, 0.1, 0.1), (0.9, 0.9, 0.9)), width=0.004, core=0.0004)
    a_side = case["x"] < 0.5
    for k in ("ax", "ay", "az"):
        case[k] = np.where(a_side, np.float32(0), case[k]).astype(np.float32)
    tg = np.nonzero(a_side)[0]
    ref = oracle.direct(case, targets=tg)["u"]
    t = vf.case_to_device(case)
    errs = []
    for p in (4, 6, 8, 10, 12):
        with vf.Context(p=p, ncrit=32, precision=2, box_lo=(0.0, 0.0, 0.0), box_len=1.0) as ctx:
            ctx.build(t[0], t[1], t[2], t[6])
            ctx.evaluate(*t)
            torch.cuda.synchronize()
            # the float64 far field (the outputs of the C ABI are float32); the
            # near field of the zero-strength cluster is zero
            fu = ctx.expansions()["far_u"]
            perm = ctx.lists()["perm"]
        u = np.empty((case["n"], 3))
        u[perm] = fu.T
        errs.append(np.abs(u[tg] - ref).max() / np.abs(ref).max())
    print("M2L chain, float64 form, p = 4 .. 12: worst particle error", ["%.1e" % e for e in errs])
    for a, b in zip(errs, errs[1:]):
        assert b <= a / 20 or b <= 1e-12
    assert errs[-1] <= 1e-12
