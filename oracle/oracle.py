"""Python access to the C oracle (ctypes), for tests and the CPU baseline.

TEST INFRASTRUCTURE ONLY: the library never imports this module.  See
``vtm_oracle.c`` for what is computed and where each step comes from in the
paper (Section 4 EVS, eq. (5.6)-(5.8) and Table 1 for VTM).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None

KIND = {"grid": 0, "rcb": 1, "graph": 2, "user": 3}
SPLIT = {"branch": 0, "equal": 1}
TOPO = {"face": 0, "complete": 1, "tree": 2}
ERR = {0: "ok", -1: "invalid", -2: "partition", -3: "not_spd", -4: "oom"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERR.get(code, '?')})")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.or_partition.restype = C.c_int
        L.or_partition.argtypes = [C.c_int64, P, P, P, C.c_int32, P, P, C.c_int32, C.c_uint64, C.c_double,
                                   C.c_double, P, C.c_int32, C.c_int32, P, P, P, P, P, C.c_int32, C.c_int32,
                                   C.c_int32, C.POINTER(C.c_void_p)]
        L.or_free.argtypes = [P]
        L.or_sizes.argtypes = [P, P]
        L.or_get.argtypes = [P] + [P] * 16
        L.or_setup.restype = C.c_int
        L.or_setup.argtypes = [P, P, C.POINTER(C.c_void_p)]
        L.or_setup_coupled.restype = C.c_int
        L.or_setup_coupled.argtypes = [P, P, C.c_int64, P, P, P, C.POINTER(C.c_void_p)]
        L.or_solver_free.argtypes = [P]
        L.or_run.restype = C.c_int64
        L.or_run.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_double, C.c_int32, P, P, P, P, P, C.c_int64]
        L.or_run_local.restype = C.c_int64
        L.or_run_local.argtypes = [P, P, P, C.c_int64, P]
        L.or_rcb_seed.restype = C.c_int64
        L.or_rcb_seed.argtypes = [P]
        L.or_num_threads.restype = C.c_int
        L.or_splitmix64_seq.argtypes = [C.c_uint64, C.c_int32, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def splitmix64_seq(seed: int, n: int) -> list[int]:
    out = np.zeros(n, dtype=np.uint64)
    lib().or_splitmix64_seq(seed, n, _p(out))
    return [int(v) for v in out]


def num_threads() -> int:
    return int(lib().or_num_threads())


class Partition:
    """EVS partition computed by the oracle; all arrays are NumPy copies."""

    def __init__(self, A, spec: dict, split: str = "branch", topology: str = "face"):
        L = lib()
        self.A = A
        rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        col = np.ascontiguousarray(A.col, dtype=np.int32)
        val = np.ascontiguousarray(A.val, dtype=np.float64)
        kind = spec["kind"]
        dims = np.array(list(spec.get("dims", (1, 1, 1))) + [1] * (3 - len(spec.get("dims", (1, 1, 1)))), dtype=np.int32)
        parts = np.array(list(spec.get("parts", (1, 1, 1))) + [1] * (3 - len(spec.get("parts", (1, 1, 1)))), dtype=np.int32)
        levels = int(spec.get("levels", 0))
        seed = int(spec.get("seed", 0))
        mn = float(spec.get("min_size", 0.0))
        mx = float(spec.get("max_size", np.inf))
        coords = spec.get("coords")
        coords = None if coords is None else np.ascontiguousarray(coords, dtype=np.float64)
        dim = 0 if coords is None else int(coords.shape[1])
        blocks = spec.get("blocks", [])
        bstart = np.array([b[0] for b in blocks], dtype=np.int64)
        bcount = np.array([b[1] for b in blocks], dtype=np.int64)
        bparts = np.array([b[2] for b in blocks], dtype=np.int32)
        usp = spec.get("s_ptr")
        usi = spec.get("s_idx")
        usp = None if usp is None else np.ascontiguousarray(usp, dtype=np.int64)
        usi = None if usi is None else np.ascontiguousarray(usi, dtype=np.int32)
        unsub = int(spec.get("nsub", 0))
        h = C.c_void_p()
        rc = L.or_partition(A.n, _p(rowptr), _p(col), _p(val), KIND[kind], _p(dims), _p(parts), levels, seed, mn, mx,
                            _p(coords), dim, len(blocks), _p(bstart), _p(bcount), _p(bparts), _p(usp), _p(usi), unsub,
                            SPLIT[split], TOPO[spec.get("topology", topology)], C.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h
        self.rcb_seed = int(L.or_rcb_seed(h))
        sz = np.zeros(7, dtype=np.int64)
        L.or_sizes(h, _p(sz))
        n, nsub, nsplit, nloc, nvtl, nports, ns = (int(v) for v in sz)
        self.n, self.nsub, self.nsplit, self.nvtl, self.nports = n, nsub, nsplit, nvtl, nports
        self.s_ptr = np.zeros(n + 1, np.int64)
        self.s_idx = np.zeros(ns, np.int32)
        self.loc_ptr = np.zeros(nsub + 1, np.int64)
        self.loc_vtx = np.zeros(nsplit, np.int64)
        self.lrp = np.zeros(nsplit + 1, np.int64)
        self.lcol = np.zeros(nloc, np.int32)
        self.lval = np.zeros(nloc, np.float64)
        self.vtl_v = np.zeros(nvtl, np.int64)
        self.vtl_k = np.zeros(nvtl, np.int32)
        self.vtl_k2 = np.zeros(nvtl, np.int32)
        self.port_ptr = np.zeros(nsub + 1, np.int64)
        self.port_v = np.zeros(nports, np.int64)
        self.port_other = np.zeros(nports, np.int32)
        self.port_twin = np.zeros(nports, np.int64)
        self.port_vtl = np.zeros(nports, np.int64)
        self.zdiag = np.zeros(nvtl, np.float64)
        L.or_get(h, *(_p(a) for a in (self.s_ptr, self.s_idx, self.loc_ptr, self.loc_vtx, self.lrp, self.lcol,
                                       self.lval, self.vtl_v, self.vtl_k, self.vtl_k2, self.port_ptr, self.port_v,
                                       self.port_other, self.port_twin, self.port_vtl, self.zdiag)))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_free(self._h)
            self._h = None

    def local_dense(self, k: int) -> np.ndarray:
        """Dense split piece A~_k over the subdomain's sorted local vertices."""
        b, e = self.loc_ptr[k], self.loc_ptr[k + 1]
        nk = int(e - b)
        a = np.zeros((nk, nk))
        for i in range(nk):
            s, t = self.lrp[b + i], self.lrp[b + i + 1]
            a[i, self.lcol[s:t]] = self.lval[s:t]
        return a

    def multiplicity(self) -> np.ndarray:
        return np.diff(self.s_ptr)


class Solver:
    """Port-augmented local factors for a given Z per VTL, and the VTM iteration.

    coupling = (l1, l2, zc): off-diagonal entries Z[l1[e]][l2[e]] = zc[e] of a symmetric impedance
    matrix over the VTLs (coupled VTLs, Section 7.2), z_vtl its diagonal; coupled VTLs join the same
    two subgraphs."""

    def __init__(self, part: Partition, z_vtl: np.ndarray, coupling=None):
        self.part = part
        z = np.ascontiguousarray(z_vtl, dtype=np.float64)
        if z.shape[0] != part.nvtl:
            raise ValueError("z_vtl must have one value per VTL")
        h = C.c_void_p()
        if coupling is not None:
            l1 = np.ascontiguousarray(coupling[0], dtype=np.int64)
            l2 = np.ascontiguousarray(coupling[1], dtype=np.int64)
            zc = np.ascontiguousarray(coupling[2], dtype=np.float64)
            rc = lib().or_setup_coupled(part._h, _p(z), len(l1), _p(l1), _p(l2), _p(zc), C.byref(h))
        else:
            rc = lib().or_setup(part._h, _p(z), C.byref(h))
        self._h = h
        if rc != 0:
            raise OracleError(rc)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_solver_free(self._h)
            self._h = None

    def run(self, b: np.ndarray, max_sweeps: int, check_every: int = 1, tol: float = 0.0, sys_ptr=None,
            waves: np.ndarray | None = None, hist_cap: int = 0):
        """Run VTM on each right-hand side (rows of b).  Returns a dict with the merged
        potentials x (nrhs, n), iters (nrhs, nsys), relres (nrhs, nsys), sweeps per RHS,
        the final incoming waves (nrhs, nports) and optional residual history."""
        b = np.atleast_2d(np.asarray(b, dtype=np.float64))
        p = self.part
        if sys_ptr is None:
            sys_ptr = np.array([0, p.n], dtype=np.int64)
        sys_ptr = np.ascontiguousarray(sys_ptr, dtype=np.int64)
        nsys = sys_ptr.shape[0] - 1
        nr = b.shape[0]
        x = np.zeros((nr, p.n))
        iters = np.zeros((nr, nsys), np.int64)
        rel = np.zeros((nr, nsys))
        sweeps = np.zeros(nr, np.int64)
        wout = np.zeros((nr, p.nports))
        hist = np.zeros((nr, max(hist_cap, 1)))
        for r in range(nr):
            bb = np.ascontiguousarray(b[r])
            a = np.zeros(p.nports) if waves is None else np.array(waves[r], dtype=np.float64)
            xr = np.zeros(p.n)
            it = np.zeros(nsys, np.int64)
            rr = np.zeros(nsys)
            hr = np.zeros(max(hist_cap, 1))
            sweeps[r] = lib().or_run(self._h, _p(bb), _p(a), int(max_sweeps), int(check_every), float(tol), nsys,
                                     _p(sys_ptr), _p(xr), _p(it), _p(rr), _p(hr) if hist_cap else None, int(hist_cap))
            x[r], iters[r], rel[r], wout[r], hist[r] = xr, it, rr, a, hr
        return dict(x=x, iters=iters, relres=rel, sweeps=sweeps, waves=wout, hist=hist[:, :hist_cap])

    def run_local(self, b: np.ndarray, nsweeps: int, waves: np.ndarray | None = None):
        """Local solutions x_k (concatenated in subdomain order) after nsweeps, and waves."""
        p = self.part
        bb = np.ascontiguousarray(b, dtype=np.float64)
        a = np.zeros(p.nports) if waves is None else np.array(waves, dtype=np.float64)
        xl = np.zeros(p.nsplit)
        lib().or_run_local(self._h, _p(bb), _p(a), int(nsweeps), _p(xl))
        return xl, a
