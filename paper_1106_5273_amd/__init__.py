"""MI355X vortex-particle FMM: Python binding of the C ABI in include/vfmm.h.

This module only marshals arguments: it passes device pointers of torch CUDA
tensors and the current HIP stream to libvfmm.so (built in-tree by
``paper_1106_5273_amd.build``).  Every step of the computation runs in the
library's HIP kernels.  If the library is missing this import fails loudly;
there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvfmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libvfmm.so not found at %s: build it with `python -m paper_1106_5273_amd.build` "
                      "(or __graft_entry__.build())" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

VFMM_OK = 0
STATUS = {0: "VFMM_OK", -1: "VFMM_EINVAL", -2: "VFMM_ENOMEM", -3: "VFMM_EDEPTH", -4: "VFMM_EDOMAIN",
          -5: "VFMM_ESTATE", -6: "VFMM_EHIP"}
SCHEME_TRANSPOSE = 0
SCHEME_CLASSICAL = 1


class Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("ncrit", ctypes.c_int32), ("theta", ctypes.c_float),
                ("sigma_gap", ctypes.c_float), ("periodic", ctypes.c_int32), ("images", ctypes.c_int32),
                ("box_lo", ctypes.c_double * 3), ("box_len", ctypes.c_double), ("scheme", ctypes.c_int32),
                ("kahan", ctypes.c_int32), ("zero_mean", ctypes.c_int32), ("direct", ctypes.c_int32),
                ("m2l_mode", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("m2l_form", ctypes.c_int32)]


class Timings(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("bounds_sort_ms", "tree_ms", "traverse_ms", "p2m_m2m_ms",
                                               "lattice_ms", "m2l_ms", "l2l_l2p_ms", "p2p_ms", "build_ms",
                                               "evaluate_ms")]


class TuneResult(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("theta", ctypes.c_float), ("ncrit", ctypes.c_int32),
                ("sigma_gap", ctypes.c_float), ("precision", ctypes.c_int32), ("m2l_form", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("err_u", ctypes.c_float), ("err_dalpha", ctypes.c_float),
                ("worst_u", ctypes.c_float), ("worst_dalpha", ctypes.c_float), ("ms", ctypes.c_float),
                ("tried", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


class RbfInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 3), ("matvecs", ctypes.c_int32), ("residual", ctypes.c_double * 3),
                ("pairs", ctypes.c_int64), ("solve_ms", ctypes.c_float), ("matvec_ms", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int32), ("nleaves", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("p2p_entries", ctypes.c_int32), ("p2p_pairs", ctypes.c_int64),
                ("m2l_entries", ctypes.c_int64), ("p2p_blocks", ctypes.c_int32),
                ("images_traversed", ctypes.c_int32), ("sum_alpha", ctypes.c_double * 3),
                ("sigma_min", ctypes.c_double), ("sigma_max", ctypes.c_double), ("m2l_keys", ctypes.c_int32),
                ("m2l_groups", ctypes.c_int32), ("m2l_items", ctypes.c_int32), ("m2l_split", ctypes.c_int32),
                ("stale", ctypes.c_int32), ("overfull_leaves", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_lib.vfmm_default_params.argtypes = [ctypes.POINTER(Params)]
_lib.vfmm_default_params.restype = None
_lib.vfmm_create.argtypes = [ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]
_lib.vfmm_set_params.argtypes = [_vp, ctypes.POINTER(Params)]
_lib.fmm_build.argtypes = [_vp, _i64] + [_vp] * 4
_lib.fmm_evaluate.argtypes = [_vp, _i64] + [_vp] * 13
_lib.rk_step.argtypes = [_vp, _i64, ctypes.c_float, ctypes.c_float] + [_vp] * 7
_lib.vfmm_autotune.argtypes = [_vp, _i64] + [_vp] * 7 + [ctypes.c_float, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
_lib.fmm_build_batched.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)] + [_vp] * 4
_lib.fmm_evaluate_batched.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)] + [_vp] * 13
_lib.fmm_build_targets.argtypes = [_vp, _i64] + [_vp] * 4 + [_i64] + [_vp] * 3
_lib.fmm_evaluate_targets.argtypes = [_vp, _i64] + [_vp] * 3 + [_i64] + [_vp] * 9
_lib.fmm_direct_static.argtypes = [_vp, _i64] + [_vp] * 13
_lib.fmm_gaussian_sum.argtypes = [_vp, _i64] + [_vp] * 6
_lib.rbf_reinit.argtypes = [_vp, _i64] + [_vp] * 6 + [ctypes.c_double, ctypes.c_int32, ctypes.POINTER(RbfInfo)]
_lib.vfmm_get_gaussian_ms.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
_lib.vfmm_energy_spectrum.argtypes = [_vp, ctypes.c_int32] + [_vp] * 3 + [ctypes.POINTER(ctypes.c_double)]
_lib.vfmm_get_timings.argtypes = [_vp, ctypes.POINTER(Timings)]
_lib.vfmm_get_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
_lib.vfmm_copy_lists.argtypes = [_vp] + [_i32p] * 9
_f64p = ctypes.POINTER(ctypes.c_double)
_lib.vfmm_copy_expansions.argtypes = [_vp] + [_i32p] * 4 + [_f64p] * 5
_lib.vfmm_last_error.argtypes = [_vp]
_lib.vfmm_last_error.restype = ctypes.c_char_p
_lib.vfmm_destroy.argtypes = [_vp]
_lib.vfmm_destroy.restype = None
for _f in ("vfmm_create", "vfmm_set_params", "fmm_build", "fmm_evaluate", "rk_step", "vfmm_get_timings",
           "vfmm_get_stats", "vfmm_copy_lists", "fmm_build_batched", "fmm_evaluate_batched", "vfmm_autotune",
           "fmm_build_targets", "fmm_evaluate_targets", "fmm_direct_static", "fmm_gaussian_sum", "rbf_reinit",
           "vfmm_get_gaussian_ms", "vfmm_energy_spectrum", "vfmm_copy_expansions"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("vfmm_default_params", "vfmm_create", "vfmm_set_params", "fmm_build", "fmm_evaluate", "rk_step",
            "vfmm_get_timings", "vfmm_get_stats", "vfmm_copy_lists", "vfmm_last_error", "vfmm_destroy",
            "fmm_build_batched", "fmm_evaluate_batched", "vfmm_autotune", "fmm_build_targets",
            "fmm_evaluate_targets", "fmm_direct_static", "fmm_gaussian_sum", "rbf_reinit", "vfmm_get_gaussian_ms",
            "vfmm_energy_spectrum", "vfmm_copy_expansions")
STATIC_MAX_N = 65536  # VFMM_STATIC_MAX_N


class VfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def default_params(**kw):
    p = Params()
    _lib.vfmm_default_params(ctypes.byref(p))
    names = {f for f, _ in Params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError("unknown vfmm parameter %r" % k)
        if k == "box_lo":
            for d in range(3):
                p.box_lo[d] = float(v[d])
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_tensor(t, n, name):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous float32 CUDA tensor of %d elements" % (name, n))


class Context:
    """Owns one vfmm_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, params=None, stream=None, **kw):
        import torch
        if params is None:
            params = default_params(**kw)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = _lib.vfmm_create(ctypes.byref(params), ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        if st != VFMM_OK:
            raise VfmmError(st, _lib.vfmm_last_error(None).decode())
        self._h = h
        self.params = params
        self._targets = (0, 0)

    def _raise(self, st):
        if st != VFMM_OK:
            raise VfmmError(st, _lib.vfmm_last_error(self._h).decode())

    def set_params(self, params=None, **kw):
        if params is None:
            params = default_params(**kw)
        self._raise(_lib.vfmm_set_params(self._h, ctypes.byref(params)))
        self.params = params

    def build(self, x, y, z, sigma):
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        self._raise(_lib.fmm_build(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(sigma)))

    def build_batched(self, offsets, x, y, z, sigma):
        """offsets: host sequence of nprob+1 int64 (problem b owns [offsets[b], offsets[b+1]))."""
        import numpy as np
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n = int(off[-1])
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        self._raise(_lib.fmm_build_batched(self._h, off.size - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           _ptr(x), _ptr(y), _ptr(z), _ptr(sigma)))

    def evaluate(self, x, y, z, ax, ay, az, sigma, out=None):
        """Returns (ux, uy, uz, dax, day, daz) as new tensors unless ``out`` is given."""
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (ax, "ax"), (ay, "ay"), (az, "az"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=x.device) for _ in range(6))
        args = [_ptr(t) for t in (x, y, z, ax, ay, az, sigma)] + [_ptr(t) for t in out]
        self._raise(_lib.fmm_evaluate(self._h, n, *args))
        return out

    def direct_static(self, x, y, z, ax, ay, az, sigma, out=None):
        """fmm_direct_static: the all-pairs evaluation without device allocation
        in the library (n <= STATIC_MAX_N).  Returns the six outputs."""
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (ax, "ax"), (ay, "ay"), (az, "az"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=x.device) for _ in range(6))
        args = [_ptr(t) for t in (x, y, z, ax, ay, az, sigma)] + [_ptr(t) for t in out]
        self._raise(_lib.fmm_direct_static(self._h, n, *args))
        return out

    def gaussian_sum(self, gx, gy, gz, out=None):
        """fmm_gaussian_sum on the particles of the last build: returns (wx, wy, wz)."""
        import torch
        n = gx.numel()
        for t, nm in ((gx, "gx"), (gy, "gy"), (gz, "gz")):
            _check_tensor(t, n, nm)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=gx.device) for _ in range(3))
        self._raise(_lib.fmm_gaussian_sum(self._h, n, _ptr(gx), _ptr(gy), _ptr(gz), *[_ptr(t) for t in out]))
        return out

    def gaussian_ms(self):
        ms = ctypes.c_float()
        self._raise(_lib.vfmm_get_gaussian_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def rbf_reinit(self, wx, wy, wz, tol=1e-4, maxiter=200, out=None):
        """rbf_reinit on the particles of the last build: returns ((gx, gy, gz), info dict)."""
        import torch
        n = wx.numel()
        for t, nm in ((wx, "wx"), (wy, "wy"), (wz, "wz")):
            _check_tensor(t, n, nm)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=wx.device) for _ in range(3))
        info = RbfInfo()
        self._raise(_lib.rbf_reinit(self._h, n, _ptr(wx), _ptr(wy), _ptr(wz), *[_ptr(t) for t in out],
                                    float(tol), int(maxiter), ctypes.byref(info)))
        d = {f: getattr(info, f) for f, _ in RbfInfo._fields_}
        d["iterations"] = tuple(info.iterations)
        d["residual"] = tuple(info.residual)
        return out, d

    def energy_spectrum(self, n, ux, uy, uz):
        """vfmm_energy_spectrum of a velocity on an n^3 lattice: numpy float64 E[k]."""
        import numpy as np
        for t, nm in ((ux, "ux"), (uy, "uy"), (uz, "uz")):
            _check_tensor(t, n ** 3, nm)
        E = np.zeros(int(np.rint(np.sqrt(3.0) * n / 2)) + 1, dtype=np.float64)
        self._raise(_lib.vfmm_energy_spectrum(self._h, int(n), _ptr(ux), _ptr(uy), _ptr(uz),
                                              E.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return E

    def build_targets(self, x, y, z, sigma, tx, ty, tz):
        """One tree over the particles and the target points (which carry no strength)."""
        n, m = x.numel(), tx.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        for t, nm in ((tx, "tx"), (ty, "ty"), (tz, "tz")):
            _check_tensor(t, m, nm)
        self._raise(_lib.fmm_build_targets(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(sigma), m, _ptr(tx),
                                           _ptr(ty), _ptr(tz)))
        self._targets = (n, m)

    def evaluate_targets(self, ax, ay, az, out=None):
        """Returns (ux, uy, uz, dax, day, daz) at the particles and (tux, tuy, tuz) at the targets."""
        import torch
        n, m = self._targets
        for t, nm in ((ax, "ax"), (ay, "ay"), (az, "az")):
            _check_tensor(t, n, nm)
        if out is None:
            out = tuple(torch.empty(n if k < 6 else m, dtype=torch.float32, device=ax.device) for k in range(9))
        self._raise(_lib.fmm_evaluate_targets(self._h, n, _ptr(ax), _ptr(ay), _ptr(az), m,
                                              *[_ptr(t) for t in out]))
        return out

    def rk_step(self, dt, nu, x, y, z, ax, ay, az, sigma):
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (ax, "ax"), (ay, "ay"), (az, "az"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        self._raise(_lib.rk_step(self._h, n, float(dt), float(nu), *[_ptr(t) for t in (x, y, z, ax, ay, az, sigma)]))

    def autotune(self, x, y, z, ax, ay, az, sigma, max_rel_l2=1e-4, cache_path=None):
        """Runs vfmm_autotune; the context keeps the chosen parameters.  Returns a dict."""
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (ax, "ax"), (ay, "ay"), (az, "az"), (sigma, "sigma")):
            _check_tensor(t, n, nm)
        r = TuneResult()
        cp = cache_path.encode() if cache_path else None
        self._raise(_lib.vfmm_autotune(self._h, n, *[_ptr(t) for t in (x, y, z, ax, ay, az, sigma)],
                                       float(max_rel_l2), cp, ctypes.byref(r)))
        self.params.p, self.params.theta, self.params.ncrit = r.p, r.theta, r.ncrit
        self.params.sigma_gap = r.sigma_gap
        self.params.precision, self.params.m2l_form, self.params.overlap = r.precision, r.m2l_form, r.overlap
        return {f: getattr(r, f) for f, _ in TuneResult._fields_}

    def timings(self):
        t = Timings()
        self._raise(_lib.vfmm_get_timings(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Timings._fields_}

    def stats(self):
        s = Stats()
        self._raise(_lib.vfmm_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in Stats._fields_}
        d["sum_alpha"] = tuple(s.sum_alpha)
        return d

    def lists(self):
        """Host copies of the interaction lists (numpy int32 arrays)."""
        import numpy as np
        st = self.stats()
        nc, npp, nm, n = st["ncells"], st["p2p_entries"], st["m2l_entries"], st["n"]
        a = {k: np.zeros(sz, dtype=np.int32) for k, sz in (("p2p_tgt", npp), ("p2p_src", npp), ("p2p_img", npp),
                                                            ("m2l_tgt", nm), ("m2l_src", nm), ("m2l_img", nm),
                                                            ("cell_start", nc), ("cell_count", nc), ("perm", n))}
        ptrs = [a[k].ctypes.data_as(_i32p) for k in ("p2p_tgt", "p2p_src", "p2p_img", "m2l_tgt", "m2l_src",
                                                     "m2l_img", "cell_start", "cell_count", "perm")]
        self._raise(_lib.vfmm_copy_lists(self._h, *ptrs))
        return a

    def expansions(self):
        """Host copies of the tree and its expansions after an evaluation (numpy):
        level, parent, first_child, nchild (int32[ncells]); geo (ncells, 5):
        centre, side, radius; mult, loc complex (ncells, 3, (p+1)(p+2)/2);
        far_u, far_da (3, n) in sorted order."""
        import numpy as np
        st = self.stats()
        nc, n, p = st["ncells"], st["n"], self.params.p
        ncp = (p + 1) * (p + 2) // 2
        a = {k: np.zeros(nc, dtype=np.int32) for k in ("level", "parent", "first_child", "nchild")}
        geo = np.zeros((nc, 5))
        mult = np.zeros((nc, 3, ncp, 2))
        loc = np.zeros((nc, 3, ncp, 2))
        fu = np.zeros((3, n))
        fd = np.zeros((3, n))
        ptrs = [a[k].ctypes.data_as(_i32p) for k in ("level", "parent", "first_child", "nchild")]
        ptrs += [x.ctypes.data_as(_f64p) for x in (geo, mult, loc, fu, fd)]
        self._raise(_lib.vfmm_copy_expansions(self._h, *ptrs))
        a.update(geo=geo, mult=mult[..., 0] + 1j * mult[..., 1], loc=loc[..., 0] + 1j * loc[..., 1], far_u=fu,
                 far_da=fd)
        return a

    def close(self):
        if getattr(self, "_h", None):
            _lib.vfmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def case_to_device(case, device="cuda"):
    """float32 SoA arrays of a workload dict -> tuple of CUDA tensors (x, y, z, ax, ay, az, sigma)."""
    import torch
    return tuple(torch.from_numpy(case[k]).to(device) for k in ("x", "y", "z", "ax", "ay", "az", "sigma"))
