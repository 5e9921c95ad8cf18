"""Dense NumPy forms of the paper's worked examples, for tiny systems only.

TEST INFRASTRUCTURE ONLY.  These functions restate, with dense matrices,
the pieces of the method that the paper works through by hand:
  * the split system of Example 4.1 / 4.2 (eq. (4.1), (4.2)) with the paper's
    own non-uniform shares,
  * the port-augmented local systems (5.4), (5.5) of Example 5.1 and the VTM
    iteration of Table 1,
  * the input impedance of a port (Definition 7.1, Example 7.1),
  * the iteration with coupled VTLs (Section 7.2), through the unreduced block
    system (5.7),
  * a brute-force dense Cholesky solve of the whole system.
"""
from __future__ import annotations

import numpy as np


def dense_cholesky_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b through the Cholesky factor A = L L^T (library factorisation)."""
    L = np.linalg.cholesky(A)
    y = np.linalg.solve(L, b)
    return np.linalg.solve(L.T, y)


class SplitSystem:
    """A system split by EVS into dense pieces with ports.

    pieces[k] = dict(glob=[global ids], A=dense A~_k, b=dense b~_k)
    vtls      = list of (k, i_local, k2, i2_local) pairs of twin ports
    """

    def __init__(self, n, pieces, vtls):
        self.n = n
        self.pieces = pieces
        self.vtls = vtls

    def scatter_back(self):
        """Sum of the pieces scattered into the original index space (Theorem 4.1, (A2.3))."""
        A = np.zeros((self.n, self.n))
        b = np.zeros(self.n)
        for pc in self.pieces:
            g = np.asarray(pc["glob"])
            A[np.ix_(g, g)] += pc["A"]
            b[g] += pc["b"]
        return A, b

    def ports(self, z):
        """Per subdomain: list of (local index, vtl id, impedance, side)."""
        out = [[] for _ in self.pieces]
        for l, (k, i, k2, i2) in enumerate(self.vtls):
            out[k].append((i, l, z[l], 0))
            out[k2].append((i2, l, z[l], 1))
        return out

    def augmented(self, z):
        """Port-augmented local matrices C_j + Z_j^{-1} of (5.8)."""
        mats = [pc["A"].copy() for pc in self.pieces]
        for k, plist in enumerate(self.ports(z)):
            for i, _, zz, _ in plist:
                mats[k][i, i] += 1.0 / zz
        return mats

    def vtm(self, z, sweeps, u0=None, w0=None):
        """Run the VTM iteration (5.6)-(5.8) from zero boundary variables.

        Keeps potentials u and inflow currents w of every port as in Example 5.1.
        Returns the merged solution history (mean of the children) and the final
        (u, w) per VTL end.
        """
        z = np.asarray(z, dtype=np.float64)
        nl = len(self.vtls)
        u = np.zeros((nl, 2)) if u0 is None else np.array(u0, dtype=np.float64)
        w = np.zeros((nl, 2)) if w0 is None else np.array(w0, dtype=np.float64)
        mats = self.augmented(z)
        plist = self.ports(z)
        hist = []
        for _ in range(sweeps):
            un = np.zeros_like(u)
            wn = np.zeros_like(w)
            xs = []
            for k, pc in enumerate(self.pieces):
                rhs = pc["b"].copy()
                for i, l, zz, side in plist[k]:
                    other = 1 - side
                    rhs[i] += (u[l, other] - zz * w[l, other]) / zz  # f + Z^{-1}(u_twin - Z w_twin)
                xk = np.linalg.solve(mats[k], rhs)
                xs.append(xk)
                for i, l, zz, side in plist[k]:
                    other = 1 - side
                    un[l, side] = xk[i]
                    wn[l, side] = -xk[i] / zz + u[l, other] / zz - w[l, other]  # current below (5.8)
            u, w = un, wn
            xbar = np.zeros(self.n)
            cnt = np.zeros(self.n)
            for k, pc in enumerate(self.pieces):
                g = np.asarray(pc["glob"])
                xbar[g] += xs[k]
                cnt[g] += 1
            hist.append(xbar / cnt)
        return np.array(hist), u, w, xs


    def vtm_coupled(self, Zv, sweeps):
        """VTM with coupled VTLs (Section 7.2): Zv is a symmetric SPD matrix over the VTLs, block diagonal
        over VTLs that join the same two subgraphs; subgraph k uses Z_k = Zv restricted to its ports'
        VTLs, in its port order.  Every sweep solves the block system (5.7) of each subgraph as written,

            [ A_k  -E ] [x]   [ b_k                  ]
            [ E^T  Z_k] [w] = [ u_twin - Z_k w_twin  ],

        with E the unit columns of the port vertices, so Z_k is never inverted.  Returns the merged
        solution history and the final (u, w) per VTL end."""
        Zv = np.asarray(Zv, dtype=np.float64)
        nl = len(self.vtls)
        u = np.zeros((nl, 2))
        w = np.zeros((nl, 2))
        plist = self.ports(np.diag(Zv))
        hist = []
        for _ in range(sweeps):
            un = np.zeros_like(u)
            wn = np.zeros_like(w)
            xs = []
            for k, pc in enumerate(self.pieces):
                nk, m = pc["A"].shape[0], len(plist[k])
                ls = [l for _, l, _, _ in plist[k]]
                Zk = Zv[np.ix_(ls, ls)]
                E = np.zeros((nk, m))
                for j, (i, _, _, _) in enumerate(plist[k]):
                    E[i, j] = 1.0
                M = np.block([[pc["A"], -E], [E.T, Zk]])
                ut = np.array([u[l, 1 - side] for _, l, _, side in plist[k]])
                wt = np.array([w[l, 1 - side] for _, l, _, side in plist[k]])
                sol = np.linalg.solve(M, np.concatenate([pc["b"], ut - Zk @ wt]))
                xk, wk = sol[:nk], sol[nk:]
                xs.append(xk)
                for j, (i, l, _, side) in enumerate(plist[k]):
                    un[l, side] = xk[i]
                    wn[l, side] = wk[j]
            u, w = un, wn
            xbar = np.zeros(self.n)
            cnt = np.zeros(self.n)
            for k, pc in enumerate(self.pieces):
                g = np.asarray(pc["glob"])
                xbar[g] += xs[k]
                cnt[g] += 1
            hist.append(xbar / cnt)
        return np.array(hist), u, w


def example_41():
    """Example 4.1: system (3.2) split at V3, V4 into (4.1) and (4.2)."""
    A1 = np.array([[6, -1, -2, 0], [-1, 7, 0, -1], [-2, 0, 4.8, -0.9], [0, -1, -0.9, 3.5]])
    b1 = np.array([1, 2, 1.6, 1.8])
    A2 = np.array([[3.2, -1.1, -1, 0], [-1.1, 5.5, 0, -3], [-1, 0, 10, -5], [0, -3, -5, 11]])
    b2 = np.array([1.4, 2.2, 5, 6])
    pieces = [dict(glob=[0, 1, 2, 3], A=A1, b=b1), dict(glob=[2, 3, 4, 5], A=A2, b=b2)]
    vtls = [(0, 2, 1, 0), (0, 3, 1, 1)]  # T3: 3a-3b, T4: 4a-4b
    return SplitSystem(6, pieces, vtls)


def input_impedance(Ak: np.ndarray, i: int) -> float:
    """Definition 7.1: potential at port i for a unit inflow current there, all else zero."""
    e = np.zeros(Ak.shape[0])
    e[i] = 1.0
    return float(np.linalg.solve(Ak, e)[i])


def from_oracle_partition(part, b: np.ndarray) -> SplitSystem:
    """Dense SplitSystem built from an oracle Partition (tiny systems only)."""
    pieces = []
    for k in range(part.nsub):
        g = part.loc_vtx[part.loc_ptr[k]:part.loc_ptr[k + 1]]
        mult = np.diff(part.s_ptr)[g]
        pieces.append(dict(glob=list(g), A=part.local_dense(k), b=b[g] / mult))
    vtls = []
    for l in range(part.nvtl):
        v, k, k2 = part.vtl_v[l], part.vtl_k[l], part.vtl_k2[l]
        gk = part.loc_vtx[part.loc_ptr[k]:part.loc_ptr[k + 1]]
        gk2 = part.loc_vtx[part.loc_ptr[k2]:part.loc_ptr[k2 + 1]]
        vtls.append((int(k), int(np.searchsorted(gk, v)), int(k2), int(np.searchsorted(gk2, v))))
    return SplitSystem(part.n, pieces, vtls)
