"""Python binding of libmbamg (argument marshalling only).

Every step of setup, V-cycle and solve runs in the HIP library; PyTorch
tensors only provide device memory and the stream.  Names follow the C-ABI in
include/mbamg.h.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbamg.so")

OK = 0
NOT_CONVERGED = 1


class MbamgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mbamg error {code}: {msg}")
        self.code = code


class Bsr(ctypes.Structure):
    _fields_ = [("n_brows", ctypes.c_int32), ("n_bcols", ctypes.c_int32), ("br", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("nnzb", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class FieldMap(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("dofs", ctypes.c_int32 * 4), ("n_vec", ctypes.c_int32 * 4)]


WEIGHT_FN = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("bgs_sweeps", ctypes.c_int32), ("inner_sweeps", ctypes.c_int32),
                ("theta", ctypes.c_double), ("max_levels", ctypes.c_int32), ("max_coarse", ctypes.c_int32),
                ("clone_aggregates", ctypes.c_int32), ("reuse_P", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("learned", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("omega_p", ctypes.c_double),
                ("judge", ctypes.c_int32), ("weight_fn", WEIGHT_FN), ("weight_ctx", ctypes.c_void_p),
                ("smoother", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("levels", ctypes.c_int32), ("used_learned", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("conv_factor", ctypes.c_double),
                ("op_complexity", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("reverted", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) for every symbol of include/mbamg.h
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
SIGNATURES = [
    ("mbamg_default_params", None, [ctypes.POINTER(Params)]),
    ("mbamg_setup", ctypes.c_int, [ctypes.POINTER(Bsr), ctypes.POINTER(FieldMap), ctypes.POINTER(Params), _P,
                                   ctypes.POINTER(_P)]),
    ("mbamg_vcycle", ctypes.c_int, [_P, _P, _P, _P]),
    ("mbamg_apply", ctypes.c_int, [_P, _P, _P, _P]),
    ("mbamg_solve", ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(Info), _P]),
    ("mbamg_get_info", ctypes.c_int, [_P, ctypes.POINTER(Info)]),
    ("mbamg_destroy", None, [_P]),
    ("mbamg_last_error", ctypes.c_char_p, []),
    ("mbamg_num_levels", ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    ("mbamg_level_nodes", ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32)]),
    ("mbamg_copy_aggregates", ctypes.c_int, [_P, _I32, _P]),
    ("mbamg_level_block_nodes", ctypes.c_int, [_P, _I32, _I32, ctypes.POINTER(_I32)]),
    ("mbamg_copy_block_aggregates", ctypes.c_int, [_P, _I32, _I32, _P]),
    ("mbamg_level_nnzb", ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_int64)]),
    ("mbamg_copy_level_block", ctypes.c_int, [_P, _I32, _I32, _I32, _P, _P, _P]),
    ("mbamg_copy_colours", ctypes.c_int, [_P, _I32, _I32, _P]),
    ("mbamg_timing_enable", ctypes.c_int, [_P, _I32]),
    ("mbamg_timing_get", ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    ("mbamg_vcycle_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    ("mbamg_level_vcycle_bytes", ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double)]),
    ("mbamg_features", ctypes.c_int, [_P, _I32, _P]),
    ("mbamg_level_weights", ctypes.c_int, [_P, _I32, _P, _P]),
    ("mbamg_mlp_forward", ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    ("mbamg_mlp_loss_grad", ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P, _P]),
    ("mbamg_mlp_loss_grad_noalloc", ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P, _P]),
    ("mbamg_mlp_adam", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, _P]),
    ("mbamg_probe", ctypes.c_int, [_P, _I32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), _P]),
    ("mbamg_set_omega", ctypes.c_int, [_P, ctypes.c_double]),
]

_lib = None


def lib():
    """Load libmbamg.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2103_07537_amd.build")
        # torch ships its own HIP runtime under the same soname; load it first so
        # the library and torch share one runtime (and one device context).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int, allow=(OK,)):
    if code not in allow:
        raise MbamgError(code, lib().mbamg_last_error().decode())
    return code


def default_params(**over) -> Params:
    p = Params()
    lib().mbamg_default_params(ctypes.byref(p))
    for k, v in over.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Hierarchy:
    """Owns an mbamg_hierarchy built from a 2x2 block system.

    ``blocks``: [[A00, A01], [A10, A11]] with row_ptr/col_idx/vals that are
    either NumPy arrays (host) or torch CUDA tensors (device).
    """

    def __init__(self, blocks, dofs, n_vec=None, params: Params | None = None, stream=None, mlp=None,
                 weights=None, **param_kw):
        """mlp: 5146 floats (network parameters, feature means, feature stds) for learned=1;
        weights: callable(level, n_agg, features[n_agg,12]) -> (omega_p, omega_s) for learned=2."""
        self._h = ctypes.c_void_p()
        self.dofs = tuple(int(d) for d in dofs)
        nb = len(self.dofs)
        self.n_blocks = nb
        self.n_nodes = int(blocks[0][0].n_brows)
        self.n_nodes1 = int(blocks[1][1].n_brows)
        self.n_dofs = sum(int(blocks[f][f].n_brows) * self.dofs[f] for f in range(nb))
        p = params if params is not None else default_params(**param_kw)
        self.params = p
        keep_alive = []
        if mlp is not None:
            arr = np.ascontiguousarray(mlp, dtype=np.float32)
            if arr.shape[0] != N_MLP_PARAMS + 24:
                raise ValueError("mlp must hold 5122 parameters and 24 normalisation values")
            keep_alive.append(arr)
            p.mlp = arr.ctypes.data
            p.learned = 1
        if weights is not None:
            errors = []

            def _cb(level, n_agg, feat_ptr, wp_ptr, ws_ptr, ctx):
                try:
                    F = np.ctypeslib.as_array(feat_ptr, shape=(n_agg * 12,)).reshape(n_agg, 12).copy()
                    wp, ws = weights(int(level), int(n_agg), F)
                    np.ctypeslib.as_array(wp_ptr, shape=(n_agg,))[:] = np.asarray(wp, dtype=np.float64)
                    np.ctypeslib.as_array(ws_ptr, shape=(n_agg,))[:] = np.asarray(ws, dtype=np.float64)
                except Exception as e:          # reported after setup returns
                    errors.append(e)
                    np.ctypeslib.as_array(ws_ptr, shape=(n_agg,))[:] = np.nan

            cb = WEIGHT_FN(_cb)
            keep_alive.append(cb)
            p.weight_fn = cb
            p.learned = 2
        fm = FieldMap()
        fm.n_blocks = nb
        for f in range(nb):
            fm.dofs[f] = self.dofs[f]
            fm.n_vec[f] = int(n_vec[f]) if n_vec else self.dofs[f] - 1
        arr = (Bsr * (nb * nb))()
        self._keep = []
        for f in range(nb):
            for g in range(nb):
                b = blocks[f][g]
                rp, ci, v = b.row_ptr, b.col_idx, b.vals
                on_dev = 0 if isinstance(rp, np.ndarray) else 1
                if on_dev:
                    ptrs = [rp.data_ptr(), ci.data_ptr(), v.data_ptr()]
                    assert rp.dtype.itemsize == 4 and ci.dtype.itemsize == 4 and v.dtype.itemsize == 8
                else:
                    rp = np.ascontiguousarray(rp, dtype=np.int32)
                    ci = np.ascontiguousarray(ci, dtype=np.int32)
                    v = np.ascontiguousarray(v, dtype=np.float64)
                    self._keep += [rp, ci, v]
                    ptrs = [rp.ctypes.data, ci.ctypes.data, v.ctypes.data]
                e = arr[f * nb + g]
                e.n_brows, e.n_bcols = int(b.n_brows), int(b.n_bcols)
                e.br, e.bc = self.dofs[f], self.dofs[g]
                e.nnzb = int(ci.shape[0])
                e.row_ptr, e.col_idx, e.vals = ptrs
                e.on_device = on_dev
        try:
            _check(lib().mbamg_setup(arr, ctypes.byref(fm), ctypes.byref(p), _stream_ptr(stream),
                                     ctypes.byref(self._h)))
        finally:
            p.weight_fn = WEIGHT_FN()
            p.mlp = None
        if weights is not None and errors:
            raise errors[0]
        self._keep = []

    def close(self):
        if self._h:
            lib().mbamg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- solve phase ---------------------------------------------------------
    def vcycle(self, r, z, stream=None):
        _check(lib().mbamg_vcycle(self._h, _ptr(r), _ptr(z), _stream_ptr(stream)))
        return z

    def apply(self, x, w, stream=None):
        _check(lib().mbamg_apply(self._h, _ptr(x), _ptr(w), _stream_ptr(stream)))
        return w

    def solve(self, b, x, rtol=1e-8, stream=None) -> dict:
        info = Info()
        code = _check(lib().mbamg_solve(self._h, _ptr(b), _ptr(x), ctypes.c_double(rtol), ctypes.byref(info),
                                        _stream_ptr(stream)), allow=(OK, NOT_CONVERGED))
        d = info.as_dict()
        d["converged"] = code == OK
        return d

    def info(self) -> dict:
        info = Info()
        _check(lib().mbamg_get_info(self._h, ctypes.byref(info)))
        return info.as_dict()

    # -- inspection ----------------------------------------------------------
    def num_levels(self) -> int:
        n = ctypes.c_int32()
        _check(lib().mbamg_num_levels(self._h, ctypes.byref(n)))
        return n.value

    def level_nodes(self, level: int) -> int:
        n = ctypes.c_int32()
        _check(lib().mbamg_level_nodes(self._h, level, ctypes.byref(n)))
        return n.value

    def block_nodes(self, level: int, f: int) -> int:
        n = ctypes.c_int32()
        _check(lib().mbamg_level_block_nodes(self._h, level, f, ctypes.byref(n)))
        return n.value

    def aggregates(self, level: int, f: int = 0) -> np.ndarray:
        a = np.zeros(self.block_nodes(level, f), dtype=np.int32)
        _check(lib().mbamg_copy_block_aggregates(self._h, level, f, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def colours(self, level: int, f: int) -> np.ndarray:
        a = np.zeros(self.block_nodes(level, f), dtype=np.int32)
        _check(lib().mbamg_copy_colours(self._h, level, f, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def level_block(self, level: int, f: int, g: int):
        n = self.block_nodes(level, f)
        nnzb = ctypes.c_int64()
        _check(lib().mbamg_level_nnzb(self._h, level, f, g, ctypes.byref(nnzb)))
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(max(nnzb.value, 1), dtype=np.int32)
        v = np.zeros(max(nnzb.value, 1) * self.dofs[f] * self.dofs[g])
        _check(lib().mbamg_copy_level_block(self._h, level, f, g, rp.ctypes.data_as(ctypes.c_void_p),
                                            ci.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p)))
        k = nnzb.value
        return rp, ci[:k], v[:k * self.dofs[f] * self.dofs[g]].reshape(k, self.dofs[f], self.dofs[g])

    # -- learned form --------------------------------------------------------
    def features(self, level: int) -> np.ndarray:
        nagg = self.level_nodes(level + 1)
        F = np.zeros((nagg, 12), dtype=np.float32)
        _check(lib().mbamg_features(self._h, level, F.ctypes.data_as(ctypes.c_void_p)))
        return F

    def level_weights(self, level: int):
        nagg = self.level_nodes(level + 1)
        wp = np.zeros(nagg)
        ws = np.zeros(nagg)
        _check(lib().mbamg_level_weights(self._h, level, wp.ctypes.data_as(ctypes.c_void_p),
                                         ws.ctypes.data_as(ctypes.c_void_p)))
        return wp, ws

    def probe(self, iters=10, seed=12345, stream=None) -> float:
        r = ctypes.c_double()
        _check(lib().mbamg_probe(self._h, iters, seed, ctypes.byref(r), _stream_ptr(stream)))
        return r.value

    def set_omega(self, omega: float):
        _check(lib().mbamg_set_omega(self._h, float(omega)))

    # -- measurement ---------------------------------------------------------
    def timing_enable(self, on=True):
        """on: False/0 off, True/1 every kind, 2 whole V-cycles only, 3 V-cycles and levels."""
        mode = int(on) if not isinstance(on, bool) else (1 if on else 0)
        _check(lib().mbamg_timing_enable(self._h, mode))

    def timing_get(self, kind: int) -> dict:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().mbamg_timing_get(self._h, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return {"launches": n.value, "total_ms": ms.value, "bytes": by.value}

    def vcycle_bytes(self) -> float:
        b = ctypes.c_double()
        _check(lib().mbamg_vcycle_bytes(self._h, ctypes.byref(b)))
        return b.value

    def level_vcycle_bytes(self, level: int):
        d, u = ctypes.c_double(), ctypes.c_double()
        _check(lib().mbamg_level_vcycle_bytes(self._h, level, ctypes.byref(d), ctypes.byref(u)))
        return d.value, u.value


N_MLP_PARAMS = 5122


def mlp_forward(params, x, out, stream=None):
    """out[n,2] = network(x[n,12]); torch device tensors (float32)."""
    _check(lib().mbamg_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(out), _stream_ptr(stream)))
    return out


def mlp_loss_grad(params, x, target, grad, loss, stream=None):
    _check(lib().mbamg_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(target), x.shape[0], _ptr(grad), _ptr(loss),
                                     _stream_ptr(stream)))
    return grad, loss


def mlp_loss_grad_noalloc(params, x, target, grad, loss, stream=None):
    _check(lib().mbamg_mlp_loss_grad_noalloc(_ptr(params), _ptr(x), _ptr(target), x.shape[0], _ptr(grad),
                                             _ptr(loss), _stream_ptr(stream)))


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().mbamg_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                                _stream_ptr(stream)))


def to_device(system, device="cuda"):
    """Copy a generator system's blocks into torch device tensors."""
    import torch

    class _B:
        pass

    nb = len(system.blocks)
    out = []
    for f in range(nb):
        row = []
        for g in range(nb):
            b = system.blocks[f][g]
            o = _B()
            o.n_brows, o.n_bcols = b.n_brows, b.n_bcols
            o.row_ptr = torch.from_numpy(np.ascontiguousarray(b.row_ptr, dtype=np.int32)).to(device)
            o.col_idx = torch.from_numpy(np.ascontiguousarray(b.col_idx, dtype=np.int32)).to(device)
            o.vals = torch.from_numpy(np.ascontiguousarray(b.vals, dtype=np.float64)).to(device)
            row.append(o)
        out.append(row)
    return out
