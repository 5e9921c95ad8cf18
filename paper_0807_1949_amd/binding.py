"""ctypes binding of libvtm (include/vtm.h).  Argument marshalling only.

Every computation happens in libvtm.so (host partitioner + HIP kernels).  If
the library has not been built, importing this module raises: there is no
Python or CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvtm.so")

VTM_OK, VTM_ERR_INVALID, VTM_ERR_PARTITION, VTM_ERR_NOT_SPD = 0, 1, 2, 3
VTM_ERR_NOT_CONVERGED, VTM_ERR_DIVERGED, VTM_ERR_STATE, VTM_ERR_HIP, VTM_ERR_OOM = 4, 5, 6, 7, 8
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "PARTITION", 3: "NOT_SPD", 4: "NOT_CONVERGED", 5: "DIVERGED",
                6: "STATE", 7: "HIP", 8: "OOM"}
VTM_FP64, VTM_FP32_IR = 0, 1
KIND = {"grid": 0, "rcb": 1, "graph": 2, "user": 3}
SPLIT = {"branch": 0, "equal": 1}
TOPO = {"face": 0, "complete": 1, "tree": 2}
VTM_Z_DIAG, VTM_Z_USER, VTM_Z_LEARNED, VTM_Z_MATCHED = 0, 1, 2, 3


class Options(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("precision", C.c_int32), ("check_every", C.c_int32),
                ("max_sweeps", C.c_int64), ("rhs_per_block", C.c_int32), ("leaf_size", C.c_int32),
                ("sweep_threads", C.c_int32), ("graph_mode", C.c_int32), ("sweep_variant", C.c_int32),
                ("sweep_mode", C.c_int32), ("persistent", C.c_int32), ("sweep_waves", C.c_int32),
                ("spin_limit", C.c_int32)]


class PartitionSpec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dims", C.c_int32 * 3), ("parts", C.c_int32 * 3), ("levels", C.c_int32),
                ("seed", C.c_uint64), ("min_size", C.c_double), ("max_size", C.c_double),
                ("coords", C.c_void_p), ("dim", C.c_int32), ("nblocks", C.c_int32), ("block_start", C.c_void_p),
                ("block_count", C.c_void_p), ("block_parts", C.c_void_p), ("s_ptr", C.c_void_p),
                ("s_idx", C.c_void_p), ("user_nsub", C.c_int32), ("split_rule", C.c_int32),
                ("topology", C.c_int32), ("nsys", C.c_int32), ("sys_ptr", C.c_void_p)]


class PartitionInfo(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("nclass", C.c_int32), ("n_split", C.c_int64), ("nvtl", C.c_int64),
                ("nports", C.c_int64), ("max_local", C.c_int32), ("nsys", C.c_int32),
                ("factor_entries", C.c_int64), ("rcb_seed", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("outer_steps", C.c_int32), ("checks", C.c_int32),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("sweep_ms", C.c_double),
                ("bytes_per_sweep", C.c_double), ("flops_per_sweep", C.c_double), ("sweep_mode", C.c_int32),
                ("persistent", C.c_int32), ("sweep_bytes", C.c_double)]


class VTMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# exported symbols declared in include/vtm.h and include/vtm_debug.h
EXPORTS = ("vtm_create", "vtm_destroy", "vtm_last_error", "vtm_evs_partition", "vtm_get_partition", "vtm_setup",
           "vtm_solve", "vtm_run_sweeps", "vtm_reset_waves", "vtm_get_waves", "vtm_set_waves", "vtm_get_stats",
           "vtm_debug_class", "vtm_zfeatures", "vtm_zmodel_load", "vtm_get_z", "vtm_input_impedance", "vtm_trainer_create",
           "vtm_trainer_destroy", "vtm_trainer_set_data", "vtm_trainer_grad", "vtm_trainer_epoch",
           "vtm_trainer_predict", "vtm_trainer_get_params", "vtm_autotune", "vtm_batch_solve",
           "vtm_setup_coupled", "vtm_input_impedance_noalloc")
NUM_FEATURES, ZMODEL_PARAMS, ZMODEL_TRAIN = 13, 5147, 5121


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libvtm.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.vtm_last_error.restype = C.c_char_p
        L.vtm_create.argtypes = [C.POINTER(Options), C.POINTER(C.c_void_p)]
        L.vtm_destroy.argtypes = [P]
        L.vtm_evs_partition.argtypes = [P, C.c_int64, P, P, P, C.POINTER(PartitionSpec), C.POINTER(PartitionInfo)]
        L.vtm_get_partition.argtypes = [P] + [P] * 15
        L.vtm_setup.argtypes = [P, C.c_int32, P]
        L.vtm_setup_coupled.argtypes = [P, P, C.c_int64, P, P, P]
        L.vtm_solve.argtypes = [P, P, C.c_int32, C.c_int64, C.c_double, P, C.c_int64, P, P]
        L.vtm_run_sweeps.argtypes = [P, P, C.c_int32, C.c_int64, C.c_int64, P, C.c_int64]
        L.vtm_reset_waves.argtypes = [P]
        L.vtm_get_waves.argtypes = [P, P, C.c_int32]
        L.vtm_set_waves.argtypes = [P, P, C.c_int32]
        L.vtm_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.vtm_debug_class.argtypes = [P, C.c_int32, P, P, P, P, P, P, P]
        L.vtm_zfeatures.argtypes = [P, P]
        L.vtm_zmodel_load.argtypes = [P, P, C.c_size_t]
        L.vtm_batch_solve.argtypes = [P, C.c_int32, P, C.c_int32, P, C.c_double, P, P, P, P]
        L.vtm_get_z.argtypes = [P, P]
        L.vtm_input_impedance.argtypes = [P, P]
        L.vtm_input_impedance_noalloc.argtypes = [P, P]
        L.vtm_trainer_create.argtypes = [C.c_int32, P, C.POINTER(C.c_void_p)]
        L.vtm_trainer_destroy.argtypes = [P]
        L.vtm_trainer_set_data.argtypes = [P, P, P, C.c_int64]
        L.vtm_trainer_grad.argtypes = [P, C.c_int64, C.c_int64, P, P]
        L.vtm_trainer_epoch.argtypes = [P, C.c_int64, C.c_float, C.c_uint64, P]
        L.vtm_trainer_predict.argtypes = [P, P, C.c_int64, P]
        L.vtm_trainer_get_params.argtypes = [P, P]
        L.vtm_autotune.argtypes = [P, C.c_int32, P]
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int32 if name != "vtm_last_error" else C.c_char_p
        _lib = L
    return _lib


def _np_ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(code, allow=()):
    if code != VTM_OK and code not in allow:
        raise VTMError(code, lib().vtm_last_error().decode())
    return code


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class VTM:
    """One libvtm handle.  Method names follow the C entry points."""

    def __init__(self, device: int = 0, precision: int = VTM_FP64, check_every: int = 0, max_sweeps: int = 100000,
                 rhs_per_block: int = 0, leaf_size: int = 0, stream: int | None = None, sweep_threads: int = 0,
                 graph_mode: int = 0, sweep_variant: int = 0, sweep_mode: int = 0, persistent: int = 0,
                 sweep_waves: int = 0, spin_limit: int = 0):
        self._h = C.c_void_p()
        o = Options()
        o.device = device
        o.stream = stream
        o.precision = precision
        o.check_every = check_every
        o.max_sweeps = max_sweeps
        o.rhs_per_block = rhs_per_block
        o.leaf_size = leaf_size
        o.sweep_threads = sweep_threads
        o.graph_mode = graph_mode
        o.sweep_variant = sweep_variant
        o.sweep_mode = sweep_mode
        o.persistent = persistent
        o.sweep_waves = sweep_waves
        o.spin_limit = spin_limit
        _check(lib().vtm_create(C.byref(o), C.byref(self._h)))
        self.precision = precision
        self.info = None
        self.n = None
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().vtm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- partition
    def evs_partition(self, A, spec: dict, split: str = "branch", topology: str = "face", nsys: int = 1,
                      sys_ptr=None) -> dict:
        rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        col = np.ascontiguousarray(A.col, dtype=np.int32)
        val = np.ascontiguousarray(A.val, dtype=np.float64)
        s = PartitionSpec()
        s.kind = KIND[spec["kind"]]
        dims = list(spec.get("dims", (1, 1, 1))) + [1] * 3
        parts = list(spec.get("parts", (1, 1, 1))) + [1] * 3
        for a in range(3):
            s.dims[a] = int(dims[a])
            s.parts[a] = int(parts[a])
        s.levels = int(spec.get("levels", 0))
        s.seed = int(spec.get("seed", 0))
        s.min_size = float(spec.get("min_size", 0.0))
        s.max_size = float(spec.get("max_size", np.inf))
        keep = []
        coords = spec.get("coords")
        if coords is not None:
            coords = np.ascontiguousarray(coords, dtype=np.float64)
            keep.append(coords)
            s.coords = coords.ctypes.data
            s.dim = coords.shape[1]
        blocks = spec.get("blocks", [])
        if blocks:
            bs = np.array([b[0] for b in blocks], np.int64)
            bc = np.array([b[1] for b in blocks], np.int64)
            bp = np.array([b[2] for b in blocks], np.int32)
            keep += [bs, bc, bp]
            s.nblocks = len(blocks)
            s.block_start, s.block_count, s.block_parts = bs.ctypes.data, bc.ctypes.data, bp.ctypes.data
        if spec["kind"] == "user":
            sp = np.ascontiguousarray(spec["s_ptr"], np.int64)
            si = np.ascontiguousarray(spec["s_idx"], np.int32)
            keep += [sp, si]
            s.s_ptr, s.s_idx, s.user_nsub = sp.ctypes.data, si.ctypes.data, int(spec["nsub"])
        s.split_rule = SPLIT[split]
        s.topology = TOPO[spec.get("topology", topology)]  # a spec may name its own
        if nsys > 1:
            sptr = np.ascontiguousarray(sys_ptr, np.int64)
            keep.append(sptr)
            s.nsys, s.sys_ptr = nsys, sptr.ctypes.data
        info = PartitionInfo()
        _check(lib().vtm_evs_partition(self._h, A.n, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val), C.byref(s),
                                       C.byref(info)))
        self.n = A.n
        self.info = {f: getattr(info, f) for f, _ in PartitionInfo._fields_}
        return self.info

    def get_partition(self) -> dict:
        i = self.info
        n = self.n
        out = dict(s_ptr=np.zeros(n + 1, np.int64), loc_ptr=np.zeros(i["nsub"] + 1, np.int64),
                   loc_vtx=np.zeros(i["n_split"], np.int64), lrp=np.zeros(i["n_split"] + 1, np.int64),
                   vtl_v=np.zeros(i["nvtl"], np.int64), vtl_k=np.zeros(i["nvtl"], np.int32),
                   vtl_k2=np.zeros(i["nvtl"], np.int32), port_ptr=np.zeros(i["nsub"] + 1, np.int64),
                   port_v=np.zeros(i["nports"], np.int64), port_other=np.zeros(i["nports"], np.int32),
                   port_twin=np.zeros(i["nports"], np.int64), zdiag=np.zeros(i["nvtl"], np.float64))
        L = lib()
        _check(L.vtm_get_partition(self._h, _np_ptr(out["s_ptr"]), None, None, None, _np_ptr(out["lrp"]),
                                   *([None] * 10)))
        out["s_idx"] = np.zeros(int(out["s_ptr"][-1]), np.int32)
        nl = int(out["lrp"][-1])
        out["lcol"] = np.zeros(nl, np.int32)
        out["lval"] = np.zeros(nl, np.float64)
        _check(L.vtm_get_partition(self._h, *(_np_ptr(out[k]) for k in (
            "s_ptr", "s_idx", "loc_ptr", "loc_vtx", "lrp", "lcol", "lval", "vtl_v", "vtl_k", "vtl_k2", "port_ptr",
            "port_v", "port_other", "port_twin", "zdiag"))))
        return out

    def debug_class(self, k: int) -> dict:
        sz = np.zeros(8, np.int64)
        L = lib()
        _check(L.vtm_debug_class(self._h, k, _np_ptr(sz), None, None, None, None, None, None))
        nk, nsn, nlev, nr, nsc = (int(v) for v in sz[:5])
        d = dict(nk=nk, nsn=nsn, nlev=nlev, nval=int(sz[5]), ws_u=int(sz[6]), cls=int(sz[7]),
                 perm=np.zeros(nk, np.int32), sn=np.zeros((nsn, 10), np.int32), lev_c0=np.zeros(nlev + 1, np.int32),
                 ridx=np.zeros(nr, np.uint16), rel=np.zeros(nr, np.uint16), sc=np.zeros((nsc, 2), np.int32))
        _check(L.vtm_debug_class(self._h, k, _np_ptr(sz), _np_ptr(d["perm"]), _np_ptr(d["sn"]), _np_ptr(d["lev_c0"]),
                                 _np_ptr(d["ridx"]), _np_ptr(d["rel"]), _np_ptr(d["sc"])))
        return d

    # ------------------------------------------------------------------ setup
    def setup(self, z_rule: int = VTM_Z_DIAG, z_vtl=None):
        z = None if z_vtl is None else np.ascontiguousarray(z_vtl, dtype=np.float64)
        _check(lib().vtm_setup(self._h, z_rule, _np_ptr(z)))

    def setup_coupled(self, z_vtl, vtl_a=(), vtl_b=(), z_ab=()):
        """Coupled VTLs: symmetric Z over the VTLs with diagonal z_vtl and Z[vtl_a[e]][vtl_b[e]] = z_ab[e]."""
        z = np.ascontiguousarray(z_vtl, dtype=np.float64)
        la = np.ascontiguousarray(vtl_a, dtype=np.int64)
        lb = np.ascontiguousarray(vtl_b, dtype=np.int64)
        zc = np.ascontiguousarray(z_ab, dtype=np.float64)
        _check(lib().vtm_setup_coupled(self._h, _np_ptr(z), len(la), _np_ptr(la), _np_ptr(lb), _np_ptr(zc)))

    # ------------------------------------------------------------------ solve
    def _vec(self, b):
        """(pointer, nrhs, ld, keepalive) of an (nrhs, n) block, numpy (host) or torch (device)."""
        if _is_torch(b):
            import torch

            if b.dim() == 1:
                b = b.unsqueeze(0)
            assert b.dtype == torch.float64 and b.is_contiguous()
            if self.n is not None and b.shape[1] != self.n:
                raise ValueError("right-hand side length differs from the partitioned system")
            if b.is_cuda:
                torch.cuda.synchronize(b.device)
            return C.c_void_p(b.data_ptr()), b.shape[0], b.shape[1], b
        b = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
        if self.n is not None and b.shape[1] != self.n:
            raise ValueError("right-hand side length differs from the partitioned system")
        return C.c_void_p(b.ctypes.data), b.shape[0], b.shape[1], b

    def _out_like(self, b, nrhs):
        if _is_torch(b):
            import torch

            return torch.empty((nrhs, b.shape[1]), dtype=torch.float64, device=b.device)
        return np.zeros((nrhs, b.shape[1]))

    def solve(self, b, tol: float, x=None, raise_on=(VTM_ERR_DIVERGED,)):
        pb, nrhs, ld, bk = self._vec(b)
        if x is None:
            x = self._out_like(bk, nrhs)
        px, _, ldx, xk = self._vec(x)
        nsys = self.info["nsys"] if self.info else 1
        iters = np.zeros(nrhs * nsys, np.int32)
        rel = np.zeros(nrhs * nsys, np.float64)
        code = lib().vtm_solve(self._h, pb, nrhs, ld, tol, px, ldx, _np_ptr(iters), _np_ptr(rel))
        if code != VTM_OK and (code in raise_on or code not in (VTM_ERR_NOT_CONVERGED, VTM_ERR_DIVERGED)):
            _check(code)
        return dict(x=xk, iters=iters.reshape(nrhs, nsys), relres=rel.reshape(nrhs, nsys), status=code)

    def run_sweeps(self, b, nsweeps: int, x=None):
        pb, nrhs, ld, bk = self._vec(b)
        if x is None:
            x = self._out_like(bk, nrhs)
        px, _, ldx, xk = self._vec(x)
        _check(lib().vtm_run_sweeps(self._h, pb, nrhs, ld, int(nsweeps), px, ldx))
        return xk

    def autotune(self, nrhs: int = 1):
        ch = np.zeros(4, np.int32)
        _check(lib().vtm_autotune(self._h, nrhs, _np_ptr(ch)))
        return dict(rhs_per_block=int(ch[0]), sweep_threads=int(ch[1]), sweep_variant=int(ch[2]),
                    sweep_mode=int(ch[3]))

    def reset_waves(self):
        _check(lib().vtm_reset_waves(self._h))

    def get_waves(self, nrhs: int = 1) -> np.ndarray:
        a = np.zeros((nrhs, self.info["nports"]))
        _check(lib().vtm_get_waves(self._h, _np_ptr(a), nrhs))
        return a

    def set_waves(self, a):
        a = np.ascontiguousarray(np.atleast_2d(a), dtype=np.float64)
        _check(lib().vtm_set_waves(self._h, _np_ptr(a), a.shape[0]))

    # ------------------------------------------------------- learned impedance
    def zfeatures(self) -> np.ndarray:
        out = np.zeros((self.info["nvtl"], NUM_FEATURES), np.float32)
        _check(lib().vtm_zfeatures(self._h, _np_ptr(out)))
        return out

    def zmodel_load(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().vtm_zmodel_load(self._h, _np_ptr(p), p.nbytes))

    def input_impedance(self) -> np.ndarray:
        """Input impedance of every port (Definition 7.1) with the other ports terminated by their Z."""
        r = np.zeros(self.info["nports"])
        _check(lib().vtm_input_impedance(self._h, _np_ptr(r)))
        return r

    def input_impedance_noalloc(self, out=None):
        """vtm_input_impedance_noalloc: the same values without any device allocation; out may be a
        preallocated host array or device tensor of nports doubles."""
        r = np.zeros(self.info["nports"]) if out is None else out
        ptr = C.c_void_p(r.data_ptr()) if _is_torch(r) else _np_ptr(r)
        _check(lib().vtm_input_impedance_noalloc(self._h, ptr))
        return r

    def get_z(self) -> np.ndarray:
        z = np.zeros(self.info["nvtl"])
        _check(lib().vtm_get_z(self._h, _np_ptr(z)))
        return z

    def get_stats(self) -> dict:
        s = Stats()
        _check(lib().vtm_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def batch_solve(handles, bs, tol: float, xs=None, raise_on=(VTM_ERR_DIVERGED,)):
    """vtm_batch_solve over independent handles: bs[i] is an (nrhs, n_i) block (numpy or torch)."""
    count = len(handles)
    hv = (C.c_void_p * count)(*[h._h.value for h in handles])
    bp, xp, keep, xk = (C.c_void_p * count)(), (C.c_void_p * count)(), [], []
    ldb = np.zeros(count, np.int64)
    ldx = np.zeros(count, np.int64)
    nrhs = None
    its, rels = [], []
    ip, rp = (C.c_void_p * count)(), (C.c_void_p * count)()
    for i, h in enumerate(handles):
        pb, nr, ld, bk = h._vec(bs[i])
        nrhs = nr if nrhs is None else nrhs
        if nr != nrhs:
            raise ValueError("every member needs the same number of right-hand sides")
        x = h._out_like(bk, nr) if xs is None else xs[i]
        px, _, lx, xkk = h._vec(x)
        bp[i], xp[i], ldb[i], ldx[i] = pb, px, ld, lx
        keep += [bk, xkk]
        xk.append(xkk)
        nsys = h.info["nsys"]
        its.append(np.zeros(nr * nsys, np.int32))
        rels.append(np.zeros(nr * nsys, np.float64))
        ip[i], rp[i] = its[-1].ctypes.data, rels[-1].ctypes.data
    code = lib().vtm_batch_solve(hv, count, bp, nrhs, _np_ptr(ldb), tol, xp, _np_ptr(ldx), ip, rp)
    if code != VTM_OK and (code in raise_on or code not in (VTM_ERR_NOT_CONVERGED, VTM_ERR_DIVERGED)):
        _check(code)
    return [dict(x=xk[i], iters=its[i].reshape(nrhs, -1), relres=rels[i].reshape(nrhs, -1), status=code)
            for i in range(count)]


class Trainer:
    """Device trainer of the impedance model (vtm_trainer_*)."""

    def __init__(self, params, device: int = 0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (ZMODEL_PARAMS,)
        self._t = C.c_void_p()
        _check(lib().vtm_trainer_create(device, _np_ptr(p), C.byref(self._t)))
        self.n = 0

    def close(self):
        if getattr(self, "_t", None) and self._t.value:
            lib().vtm_trainer_destroy(self._t)
            self._t = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, feats, labels):
        f = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        assert f.shape == (y.shape[0], NUM_FEATURES)
        _check(lib().vtm_trainer_set_data(self._t, _np_ptr(f), _np_ptr(y), y.shape[0]))
        self.n = y.shape[0]

    def grad(self, row0: int = 0, nrows: int | None = None):
        nrows = self.n - row0 if nrows is None else nrows
        g = np.zeros(ZMODEL_TRAIN, np.float32)
        loss = C.c_float()
        _check(lib().vtm_trainer_grad(self._t, row0, nrows, _np_ptr(g), C.byref(loss)))
        return g, loss.value

    def epoch(self, batch: int, lr: float, seed: int) -> float:
        loss = C.c_float()
        _check(lib().vtm_trainer_epoch(self._t, batch, lr, seed, C.byref(loss)))
        return loss.value

    def predict(self, feats) -> np.ndarray:
        f = np.ascontiguousarray(feats, dtype=np.float32)
        out = np.zeros(f.shape[0], np.float32)
        _check(lib().vtm_trainer_predict(self._t, _np_ptr(f), f.shape[0], _np_ptr(out)))
        return out

    def get_params(self) -> np.ndarray:
        p = np.zeros(ZMODEL_PARAMS, np.float32)
        _check(lib().vtm_trainer_get_params(self._t, _np_ptr(p)))
        return p
