"""ctypes binding of libmlqmc.so (the C ABI in include/mlqmc.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions carry the C names; arrays may be numpy (host memory,
io_on_device = 0) or torch CUDA tensors (device memory, io_on_device = 1;
the context then runs on torch's current stream).  A missing or unloadable
library raises immediately: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlqmc.so")
TUNING_PATH = os.path.join(HERE, "tuning.json")

MLQMC_OK, MLQMC_EINVAL, MLQMC_ENOMEM, MLQMC_EDEVICE, MLQMC_ENOCONV = 0, -1, -2, -3, -4
MLQMC_HOST_ONLY = -1  # device id of a host-only context (argument checks, no compute)
MLQMC_FP64, MLQMC_MIXED = 0, 1
FLAG_RQ_NOCONV, FLAG_LIN_NOCONV, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_WRONG_PAIR = 1, 2, 4, 8, 16
K_NONE, K_COEFF, K_APPLY, K_SMOOTH, K_COARSE, K_PRE, K_TG_LDS = 0, 1, 2, 3, 4, 5, 6

# every symbol include/mlqmc.h declares
EXPORTS = [
    "mlqmc_default_opts", "mlqmc_create", "mlqmc_create_islands", "mlqmc_destroy",
    "mlqmc_last_error",
    "mlqmc_lattice_points", "mlqmc_embedded_points", "mlqmc_coefficient",
    "mlqmc_apply_operator", "mlqmc_edge_weights", "mlqmc_prolong", "mlqmc_eig_level",
    "mlqmc_eig_level_noalloc", "mlqmc_estimate",
    "mlqmc_estimate_nested", "mlqmc_estimate_nested_extend", "mlqmc_adaptive_decide",
    "mlqmc_estimate_adaptive", "mlqmc_set_tuning",
    "mlqmc_set_timing", "mlqmc_get_timing",
]


class MlqmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mlqmc status {code}: {msg}")
        self.code = code


class Coeff(C.Structure):
    _fields_ = [("s_max", C.c_int32), ("a0", C.c_double), ("c", C.POINTER(C.c_double)),
                ("k1", C.POINTER(C.c_int32)), ("k2", C.POINTER(C.c_int32))]


class Islands(C.Structure):
    _fields_ = [("s_max", C.c_int32), ("a0_in", C.c_double), ("a0_out", C.c_double),
                ("b0_in", C.c_double), ("b0_out", C.c_double),
                ("ca", C.POINTER(C.c_double)), ("cb", C.POINTER(C.c_double)),
                ("k1", C.POINTER(C.c_int32)), ("k2", C.POINTER(C.c_int32)),
                ("region", C.POINTER(C.c_int32))]


class Level(C.Structure):
    _fields_ = [("n_fine", C.c_int32), ("s_fine", C.c_int32), ("n_coarse", C.c_int32),
                ("s_coarse", C.c_int32), ("n_prev", C.c_int32), ("s_prev", C.c_int32)]


class AdaptiveOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("alpha", C.c_double), ("gamma", C.c_double),
                ("N_init", C.c_int64), ("N_max", C.c_int64)]


ADAPT_DONE, ADAPT_DOUBLE, ADAPT_ADD, ADAPT_BUDGET, ADAPT_LEVELS = 0, 1, 2, 3, 4


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("eig_rtol", C.c_double), ("max_rq_iter", C.c_int32),
                ("lin_rtol", C.c_double), ("lam_rtol", C.c_double), ("rq_lin_rtol", C.c_double),
                ("max_lin_iter", C.c_int32), ("chain_len", C.c_int32), ("batch", C.c_int32),
                ("pcg_graph", C.c_int32), ("io_on_device", C.c_int32),
                ("device_mem_cap", C.c_int64), ("eig_atol", C.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads the library (once).  Raises if it is missing or incomplete."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2103_03407_amd.build` (no CPU fallback exists)")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # SONAME); importing torch first makes this library bind to that copy
    # instead of loading a second runtime that would not see the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name in EXPORTS:
        getattr(lib, name)  # AttributeError if absent
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.mlqmc_default_opts.argtypes = [C.POINTER(Opts)]
    lib.mlqmc_default_opts.restype = None
    lib.mlqmc_create.argtypes = [C.POINTER(P), C.POINTER(Coeff), C.c_int, P]
    lib.mlqmc_create_islands.argtypes = [C.POINTER(P), C.POINTER(Islands), C.c_int, P]
    lib.mlqmc_destroy.argtypes = [P]
    lib.mlqmc_destroy.restype = None
    lib.mlqmc_last_error.argtypes = [P]
    lib.mlqmc_last_error.restype = C.c_char_p
    lib.mlqmc_lattice_points.argtypes = [P, I64, I32, P, P, I64, I64, P, I32]
    lib.mlqmc_embedded_points.argtypes = [P, I64, I32, P, P, I64, I64, P, I32]
    lib.mlqmc_coefficient.argtypes = [P, I32, I32, I64, P, P, I32]
    lib.mlqmc_apply_operator.argtypes = [P, I32, I32, I64, P, P, P, P, I32]
    lib.mlqmc_edge_weights.argtypes = [P, I32, I32, I64, P, P, I32]
    lib.mlqmc_prolong.argtypes = [P, I32, I32, I64, P, P, I32]
    lib.mlqmc_eig_level.argtypes = [P, C.POINTER(Level), C.POINTER(Opts), I64, P, I32, P, P, P,
                                    P, P, P, P, P]
    lib.mlqmc_eig_level_noalloc.argtypes = [P, C.POINTER(Level), C.POINTER(Opts), I64, P, I32,
                                            P, P, P, P, P, P]
    lib.mlqmc_estimate.argtypes = [P, I32, C.POINTER(Level), P, I32, P, P, C.POINTER(Opts), P,
                                   P, P, P, P]
    lib.mlqmc_estimate_nested.argtypes = [P, I32, C.POINTER(Level), P, I32, P, P,
                                          C.POINTER(Opts), P, P, P, P, P, P]
    lib.mlqmc_estimate_nested_extend.argtypes = [P, I32, C.POINTER(Level), P, P, I32, P, P,
                                                 C.POINTER(Opts), P, P, P, P, P, P, P]
    lib.mlqmc_adaptive_decide.argtypes = [I32, I32, P, P, P, P, D, D, I64, C.POINTER(I32)]
    lib.mlqmc_adaptive_decide.restype = C.c_int32
    lib.mlqmc_estimate_adaptive.argtypes = [P, I32, C.POINTER(Level), I32, P, P,
                                            C.POINTER(AdaptiveOpts), C.POINTER(Opts),
                                            C.POINTER(I32), P, P, P, P, P, C.POINTER(I32), P, I32,
                                            C.POINTER(I32)]
    lib.mlqmc_set_tuning.argtypes = [P, I32, I32, I64]
    lib.mlqmc_set_timing.argtypes = [P, I32]
    lib.mlqmc_get_timing.argtypes = [P, C.POINTER(I64), C.POINTER(D), C.POINTER(D),
                                     C.POINTER(D)]
    for name in ("mlqmc_create", "mlqmc_create_islands", "mlqmc_lattice_points",
                 "mlqmc_embedded_points", "mlqmc_coefficient", "mlqmc_apply_operator",
                 "mlqmc_edge_weights", "mlqmc_prolong",
                 "mlqmc_eig_level", "mlqmc_eig_level_noalloc", "mlqmc_estimate",
                 "mlqmc_estimate_nested",
                 "mlqmc_estimate_nested_extend", "mlqmc_estimate_adaptive",
                 "mlqmc_set_tuning", "mlqmc_set_timing", "mlqmc_get_timing"):
        getattr(lib, name).restype = C.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def default_opts(**kw) -> Opts:
    o = Opts()
    load().mlqmc_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, on_device) for a numpy array or torch CUDA tensor (or None)."""
    if x is None:
        return None, None
    if _is_torch(x):
        import torch
        want = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32,
                np.uint8: torch.uint8}[dtype]
        if x.dtype != want or not x.is_contiguous() or not x.is_cuda:
            raise TypeError(f"expected a contiguous CUDA tensor of {want}")
        return C.c_void_p(x.data_ptr()), True
    if not isinstance(x, np.ndarray) or x.dtype != np.dtype(dtype) or not x.flags.c_contiguous:
        raise TypeError(f"expected a C-contiguous numpy array of {np.dtype(dtype)}")
    return C.c_void_p(x.ctypes.data), False


def _shared_rule(levels, z, shifts, R):
    """z [s_max] and shifts [R, s_max] of a nested estimate, s_max the largest
    truncation of `levels` (longer rows are cut to it)."""
    s_max = max(int(l[1]) for l in levels)
    z = np.asarray(z)
    shifts = np.asarray(shifts, dtype=np.float64).reshape(R, -1)
    if z.shape[0] < s_max or shifts.shape[1] < s_max:
        raise ValueError(f"z and the shift rows need s_max = {s_max} entries")
    return (np.ascontiguousarray(z[:s_max], dtype=np.int64),
            np.ascontiguousarray(shifts[:, :s_max]))


def _one_side(*flags):
    s = {f for f in flags if f is not None}
    if len(s) > 1:
        raise TypeError("mix of host arrays and device tensors")
    return int(s.pop()) if s else 0


class Context:
    """An mlqmc_ctx bound to one device and stream.  ``family`` is a Problem 1
    table (keys a0, c, k1, k2) or, with ``kind == "islands"``, a Problem 2 table
    (keys a0_in, a0_out, b0_in, b0_out, ca, cb, k1, k2, region)."""

    def __init__(self, family, device: int = 0, stream=None):
        lib = load()
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        k1 = np.ascontiguousarray(family["k1"], dtype=np.int32)
        k2 = np.ascontiguousarray(family["k2"], dtype=np.int32)
        islands = family.get("kind") == "islands"
        if islands:
            c = np.ascontiguousarray(family["ca"], dtype=np.float64)
            cb = np.ascontiguousarray(family["cb"], dtype=np.float64)
            rg = np.ascontiguousarray(family["region"], dtype=np.int32)
            cf = Islands(int(c.size), float(family["a0_in"]), float(family["a0_out"]),
                         float(family["b0_in"]), float(family["b0_out"]), c.ctypes.data_as(dp),
                         cb.ctypes.data_as(dp), k1.ctypes.data_as(ip), k2.ctypes.data_as(ip),
                         rg.ctypes.data_as(ip))
        else:
            c = np.ascontiguousarray(family["c"], dtype=np.float64)
            cf = Coeff(int(c.size), float(family["a0"]), c.ctypes.data_as(dp),
                       k1.ctypes.data_as(ip), k2.ctypes.data_as(ip))
        if stream is None and device != MLQMC_HOST_ONLY:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                stream = None
        h = C.c_void_p()
        create = lib.mlqmc_create_islands if islands else lib.mlqmc_create
        st = create(C.byref(h), C.byref(cf), int(device), C.c_void_p(stream or 0))
        if st != MLQMC_OK:
            raise MlqmcError(st, lib.mlqmc_last_error(None).decode())
        self._lib, self._h = lib, h
        self.s_max = int(c.size)
        self.device = int(device)

    def set_tuning(self, n_fine, prec, target_blocks):
        return self._check(self._lib.mlqmc_set_tuning(self._h, int(n_fine), int(prec),
                                                      int(target_blocks)))

    def apply_tuning(self, path=None, arch=None):
        """Applies the autotuner's table (a JSON file; by default the one
        shipped beside the library) for this device's architecture.  Returns
        the number of entries applied."""
        import json
        path = path or TUNING_PATH
        if not os.path.exists(path):
            return 0
        table = json.load(open(path))
        if arch is None:
            try:
                import torch
                arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
            except Exception:
                return 0
        count = 0
        for e in table.get(arch, []):
            prec = MLQMC_MIXED if e["prec"] == "mixed" else MLQMC_FP64
            self.set_tuning(e["n_fine"], prec, e["target_blocks"])
            count += 1
        return count

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mlqmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_noconv=False):
        if st == MLQMC_OK or (allow_noconv and st == MLQMC_ENOCONV):
            return st
        raise MlqmcError(st, self._lib.mlqmc_last_error(self._h).decode())

    # ---- components ----
    def lattice_points(self, N, z, shift, k0, count, Y):
        z = np.ascontiguousarray(z, dtype=np.int64)
        shift = np.ascontiguousarray(shift, dtype=np.float64)
        py, dy = _ptr(Y, np.float64)
        return self._check(self._lib.mlqmc_lattice_points(
            self._h, int(N), int(z.size), C.c_void_p(z.ctypes.data),
            C.c_void_p(shift.ctypes.data), int(k0), int(count), py, int(bool(dy))))

    def embedded_points(self, N, z, shift, k0, count, Y):
        z = np.ascontiguousarray(z, dtype=np.int64)
        shift = np.ascontiguousarray(shift, dtype=np.float64)
        py, dy = _ptr(Y, np.float64)
        return self._check(self._lib.mlqmc_embedded_points(
            self._h, int(N), int(z.size), C.c_void_p(z.ctypes.data),
            C.c_void_p(shift.ctypes.data), int(k0), int(count), py, int(bool(dy))))

    def coefficient(self, n, s, Y, aK):
        py, dy = _ptr(Y, np.float64)
        pa, da = _ptr(aK, np.float64)
        B = Y.shape[0]
        return self._check(self._lib.mlqmc_coefficient(self._h, int(n), int(s), int(B), py, pa,
                                                       _one_side(dy, da)))

    def apply_operator(self, n, s, Y, sigma, x, out):
        py, dy = _ptr(Y, np.float64)
        ps, ds = _ptr(sigma, np.float64)
        px, dx = _ptr(x, np.float64)
        po, do = _ptr(out, np.float64)
        B = x.shape[0]
        return self._check(self._lib.mlqmc_apply_operator(
            self._h, int(n), int(s), int(B), py, ps, px, po, _one_side(dy, ds, dx, do)))

    def edge_weights(self, n, s, Y, out):
        """Padded [WX | WY] edge weights, out [B, 2 (n+2) n] (mlqmc_edge_weights)."""
        py, dy = _ptr(Y, np.float64)
        po, do = _ptr(out, np.float64)
        return self._check(self._lib.mlqmc_edge_weights(self._h, int(n), int(s), int(out.shape[0]),
                                                        py, po, _one_side(dy, do)))

    def prolong(self, nH, nh, uH, uh):
        pu, du = _ptr(uH, np.float64)
        pv, dv = _ptr(uh, np.float64)
        return self._check(self._lib.mlqmc_prolong(self._h, int(nH), int(nh), int(uH.shape[0]),
                                                   pu, pv, _one_side(du, dv)))

    # ---- hot path ----
    def eig_level(self, level, Y, lam, flags, lam_prev=None, lam_coarse=None, rq_iters=None,
                  lin_iters=None, warm_chain=1, opts=None, g=None, g_prev=None):
        o = opts if opts is not None else default_opts()
        lv = Level(*[int(x) for x in level])
        # the library reads Y with row stride s_fine
        if len(Y.shape) != 2 or (Y.shape[1] != lv.s_fine and not (lv.s_fine == 0 and
                                                                   Y.shape[1] <= 1)):
            raise ValueError(f"Y must be [n, s_fine={lv.s_fine}] (got {tuple(Y.shape)})")
        py, d0 = _ptr(Y, np.float64)
        pl, d1 = _ptr(lam, np.float64)
        pf, d2 = _ptr(flags, np.uint8)
        pp, d3 = _ptr(lam_prev, np.float64)
        pc, d4 = _ptr(lam_coarse, np.float64)
        pr, d5 = _ptr(rq_iters, np.int32)
        pi, d6 = _ptr(lin_iters, np.int32)
        pg, d7 = _ptr(g, np.float64)
        pgp, d8 = _ptr(g_prev, np.float64)
        o.io_on_device = _one_side(d0, d1, d2, d3, d4, d5, d6, d7, d8)
        n = Y.shape[0]
        return self._check(self._lib.mlqmc_eig_level(
            self._h, C.byref(lv), C.byref(o), int(n), py, int(warm_chain), pl, pp, pc, pr, pi,
            pf, pg, pgp), allow_noconv=True)

    def eig_level_noalloc(self, level, Y, lam, flags, lam_prev=None, lam_coarse=None,
                          rq_iters=None, lin_iters=None, warm_chain=1, opts=None):
        """mlqmc_eig_level_noalloc: device tensors only (the library allocates
        nothing; meshes up to 1/32)."""
        o = opts if opts is not None else default_opts()
        lv = Level(*[int(x) for x in level])
        if len(Y.shape) != 2 or (Y.shape[1] != lv.s_fine and not (lv.s_fine == 0 and
                                                                   Y.shape[1] <= 1)):
            raise ValueError(f"Y must be [n, s_fine={lv.s_fine}] (got {tuple(Y.shape)})")
        py, d0 = _ptr(Y, np.float64)
        pl, d1 = _ptr(lam, np.float64)
        pf, d2 = _ptr(flags, np.uint8)
        pp, d3 = _ptr(lam_prev, np.float64)
        pc, d4 = _ptr(lam_coarse, np.float64)
        pr, d5 = _ptr(rq_iters, np.int32)
        pi, d6 = _ptr(lin_iters, np.int32)
        o.io_on_device = _one_side(d0, d1, d2, d3, d4, d5, d6)
        return self._check(self._lib.mlqmc_eig_level_noalloc(
            self._h, C.byref(lv), C.byref(o), int(Y.shape[0]), py, int(warm_chain), pl, pp, pc,
            pr, pi, pf), allow_noconv=True)

    def estimate_adaptive(self, levels, R, z, shifts, eps, alpha=2.0, gamma=2.0, N_init=8,
                          N_max=1 << 20, opts=None, trace_cap=256):
        """mlqmc_estimate_adaptive over the nested hierarchy `levels` (6-tuples,
        the most levels allowed).  Returns (status, dict) with n_levels, N,
        Q_lr, Qhat, V, est, converged and trace [(action, level)]."""
        o = opts if opts is not None else default_opts()
        o.io_on_device = 0
        Lm = len(levels)
        lv = (Level * Lm)(*[Level(*[int(x) for x in l]) for l in levels])
        zc, sc = _shared_rule(levels, z, shifts, R)
        ao = AdaptiveOpts(float(eps), float(alpha), float(gamma), int(N_init), int(N_max))
        nl = C.c_int32()
        conv = C.c_int32()
        tlen = C.c_int32()
        N = np.zeros(Lm, np.int64)
        Q = np.zeros((Lm, R))
        Qh, V, est = np.zeros(Lm), np.zeros(Lm), np.zeros(2)
        tr = np.zeros((trace_cap, 2), np.int32)
        st = self._check(self._lib.mlqmc_estimate_adaptive(
            self._h, Lm, lv, int(R), C.c_void_p(zc.ctypes.data), C.c_void_p(sc.ctypes.data),
            C.byref(ao), C.byref(o), C.byref(nl), C.c_void_p(N.ctypes.data),
            C.c_void_p(Q.ctypes.data), C.c_void_p(Qh.ctypes.data), C.c_void_p(V.ctypes.data),
            C.c_void_p(est.ctypes.data), C.byref(conv), C.c_void_p(tr.ctypes.data),
            int(trace_cap), C.byref(tlen)), allow_noconv=True)
        L = nl.value
        return st, {"n_levels": L, "N": N[:L].tolist(), "Q_lr": Q[:L], "Qhat": Qh[:L],
                    "V": V[:L], "est": est, "converged": bool(conv.value),
                    "trace": [tuple(int(v) for v in tr[i]) for i in range(min(tlen.value,
                                                                               trace_cap))]}

    @staticmethod
    def _g_split(G, L, R):
        Q = G[:L * R].reshape(L, R)
        return Q, G[L * R:L * R + L], G[L * R + L:L * R + 2 * L], G[L * R + 2 * L:]

    def estimate(self, levels, N, R, z, shifts, opts=None, functional=False):
        """levels: list of 6-tuples; z, shifts: per-level arrays.  Returns
        (status, Q_lr [L,R], Qhat [L], V [L], est [2]) as host arrays, and with
        functional=True a sixth item (Q_lr, Qhat, V, est) for E[G(u)]."""
        o = opts if opts is not None else default_opts()
        o.io_on_device = 0
        L = len(levels)
        lv = (Level * L)(*[Level(*[int(x) for x in l]) for l in levels])
        Nn = np.ascontiguousarray(N, dtype=np.int64)
        zc = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.int64) for a in z]))
        sc = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).ravel()
                                                  for a in shifts]))
        Q = np.zeros((L, R))
        Qh = np.zeros(L)
        V = np.zeros(L)
        est = np.zeros(2)
        G = np.zeros(L * R + 2 * L + 2) if functional else None
        st = self._check(self._lib.mlqmc_estimate(
            self._h, L, lv, C.c_void_p(Nn.ctypes.data), int(R), C.c_void_p(zc.ctypes.data),
            C.c_void_p(sc.ctypes.data), C.byref(o), C.c_void_p(Q.ctypes.data),
            C.c_void_p(Qh.ctypes.data), C.c_void_p(V.ctypes.data), C.c_void_p(est.ctypes.data),
            C.c_void_p(G.ctypes.data) if functional else None), allow_noconv=True)
        if functional:
            return st, Q, Qh, V, est, self._g_split(G, L, R)
        return st, Q, Qh, V, est

    def estimate_nested(self, levels, N, R, z, shifts, opts=None, lam_out=False,
                        functional=False):
        """Nested estimator with shared shifts: z [s_max], shifts [R, s_max].
        Returns (status, Q_lr, Qhat, V, est, lam) with lam the per-level
        lambda^l values [level][r, k] (or None), and with functional=True a
        seventh item (Q_lr, Qhat, V, est) for E[G(u)]."""
        o = opts if opts is not None else default_opts()
        o.io_on_device = 0
        L = len(levels)
        lv = (Level * L)(*[Level(*[int(x) for x in l]) for l in levels])
        Nn = np.ascontiguousarray(N, dtype=np.int64)
        zc, sc = _shared_rule(levels, z, shifts, R)
        Q = np.zeros((L, R))
        Qh = np.zeros(L)
        V = np.zeros(L)
        est = np.zeros(2)
        lo = np.zeros(int(R * Nn.sum())) if lam_out else None
        G = np.zeros(L * R + 2 * L + 2) if functional else None
        st = self._check(self._lib.mlqmc_estimate_nested(
            self._h, L, lv, C.c_void_p(Nn.ctypes.data), int(R), C.c_void_p(zc.ctypes.data),
            C.c_void_p(sc.ctypes.data), C.byref(o), C.c_void_p(Q.ctypes.data),
            C.c_void_p(Qh.ctypes.data), C.c_void_p(V.ctypes.data), C.c_void_p(est.ctypes.data),
            C.c_void_p(lo.ctypes.data) if lam_out else None,
            C.c_void_p(G.ctypes.data) if functional else None), allow_noconv=True)
        lam = None
        if lam_out:
            lam, off = [], 0
            for Nl in Nn:
                lam.append(lo[off:off + R * Nl].reshape(R, Nl))
                off += R * Nl
        if functional:
            return st, Q, Qh, V, est, lam, self._g_split(G, L, R)
        return st, Q, Qh, V, est, lam

    def estimate_nested_extend(self, levels, N_done, N, R, z, shifts, sums, opts=None,
                               g_sums=None):
        """Continues a nested estimate from N_done[l] to N[l] points per level.
        sums: float64 [L, R], updated in place (the per-(level, shift) sums of
        Y_l over the points done; zeros to start).  g_sums: the same for G, or
        None.  Returns (status, Q_lr, Qhat, V, est) and, with g_sums, a sixth
        item (Q_lr, Qhat, V, est) for E[G(u)]."""
        o = opts if opts is not None else default_opts()
        o.io_on_device = 0
        L = len(levels)
        lv = (Level * L)(*[Level(*[int(x) for x in l]) for l in levels])
        Nd = np.ascontiguousarray(N_done, dtype=np.int64)
        Nn = np.ascontiguousarray(N, dtype=np.int64)
        zc, sc = _shared_rule(levels, z, shifts, R)
        for arr in (sums, g_sums):
            if arr is not None and (not isinstance(arr, np.ndarray) or arr.dtype != np.float64
                                    or not arr.flags.c_contiguous or arr.size != L * R):
                raise TypeError("sums must be a C-contiguous float64 array of L x R entries")
        if Nd.size != L or Nn.size != L:
            raise ValueError("N_done and N need one entry per level")
        Q = np.zeros((L, R))
        Qh = np.zeros(L)
        V = np.zeros(L)
        est = np.zeros(2)
        G = np.zeros(L * R + 2 * L + 2) if g_sums is not None else None
        st = self._check(self._lib.mlqmc_estimate_nested_extend(
            self._h, L, lv, C.c_void_p(Nd.ctypes.data), C.c_void_p(Nn.ctypes.data), int(R),
            C.c_void_p(zc.ctypes.data), C.c_void_p(sc.ctypes.data), C.byref(o),
            C.c_void_p(sums.ctypes.data), C.c_void_p(Q.ctypes.data), C.c_void_p(Qh.ctypes.data),
            C.c_void_p(V.ctypes.data), C.c_void_p(est.ctypes.data),
            C.c_void_p(g_sums.ctypes.data) if g_sums is not None else None,
            C.c_void_p(G.ctypes.data) if G is not None else None), allow_noconv=True)
        if G is not None:
            return st, Q, Qh, V, est, self._g_split(G, L, R)
        return st, Q, Qh, V, est

    # ---- instrumentation ----
    def set_timing(self, kernel_class):
        return self._check(self._lib.mlqmc_set_timing(self._h, int(kernel_class)))

    def get_timing(self, flops=False):
        """(launches, total ms, model bytes[, model flops]) of the timed class."""
        n = C.c_int64()
        ms = C.c_double()
        by = C.c_double()
        fl = C.c_double()
        self._check(self._lib.mlqmc_get_timing(self._h, C.byref(n), C.byref(ms), C.byref(by),
                                               C.byref(fl)))
        if flops:
            return int(n.value), float(ms.value), float(by.value), float(fl.value)
        return int(n.value), float(ms.value), float(by.value)


# module-level functions with the C names
def mlqmc_create(family, device=0, stream=None) -> Context:
    return Context(family, device, stream)


def mlqmc_create_islands(family, device=0, stream=None) -> Context:
    if family.get("kind") != "islands":
        raise ValueError("mlqmc_create_islands takes a Problem 2 (islands) family")
    return Context(family, device, stream)


def mlqmc_destroy(ctx: Context) -> None:
    ctx.close()


def mlqmc_last_error(ctx: Context | None = None) -> str:
    lib = load()
    return lib.mlqmc_last_error(ctx._h if ctx is not None else None).decode()


def mlqmc_default_opts(**kw) -> Opts:
    return default_opts(**kw)


def mlqmc_lattice_points(ctx, *a, **k):
    return ctx.lattice_points(*a, **k)


def mlqmc_embedded_points(ctx, *a, **k):
    return ctx.embedded_points(*a, **k)


def mlqmc_estimate_nested(ctx, *a, **k):
    return ctx.estimate_nested(*a, **k)


def mlqmc_estimate_nested_extend(ctx, *a, **k):
    return ctx.estimate_nested_extend(*a, **k)


def mlqmc_coefficient(ctx, *a, **k):
    return ctx.coefficient(*a, **k)


def mlqmc_apply_operator(ctx, *a, **k):
    return ctx.apply_operator(*a, **k)


def mlqmc_edge_weights(ctx, *a, **k):
    return ctx.edge_weights(*a, **k)


def mlqmc_prolong(ctx, *a, **k):
    return ctx.prolong(*a, **k)


def mlqmc_eig_level(ctx, *a, **k):
    return ctx.eig_level(*a, **k)


def mlqmc_eig_level_noalloc(ctx, *a, **k):
    return ctx.eig_level_noalloc(*a, **k)


def mlqmc_adaptive_decide(Qhat, V, N, cost, eps, alpha, max_levels, N_max):
    """The adaptive rule's decision (host arithmetic in the library, no
    device): returns (action, level)."""
    lib = load()
    L = len(Qhat)
    q = np.ascontiguousarray(Qhat, dtype=np.float64)
    v = np.ascontiguousarray(V, dtype=np.float64)
    n = np.ascontiguousarray(N, dtype=np.int64)
    c = np.ascontiguousarray(cost, dtype=np.float64)
    lev = C.c_int32()
    act = lib.mlqmc_adaptive_decide(L, int(max_levels), C.c_void_p(q.ctypes.data),
                                    C.c_void_p(v.ctypes.data), C.c_void_p(n.ctypes.data),
                                    C.c_void_p(c.ctypes.data), float(eps), float(alpha),
                                    int(N_max), C.byref(lev))
    if act < 0:
        raise MlqmcError(MLQMC_EINVAL, "mlqmc_adaptive_decide: invalid arguments")
    return int(act), int(lev.value)


def mlqmc_estimate_adaptive(ctx, *a, **k):
    return ctx.estimate_adaptive(*a, **k)


def mlqmc_estimate(ctx, *a, **k):
    return ctx.estimate(*a, **k)


def mlqmc_set_tuning(ctx, *a, **k):
    return ctx.set_tuning(*a, **k)


def mlqmc_set_timing(ctx, *a, **k):
    return ctx.set_timing(*a, **k)


def mlqmc_get_timing(ctx):
    return ctx.get_timing()
