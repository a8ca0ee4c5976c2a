"""AlgMortar set-up and apply, FP64, following the paper step by step.

Set-up (Algorithm 1, AlgMortarSetup):
  partition -> permutation -> for each subdomain: extract ``A_ii`` and modify
  its diagonal to get ``A_i`` (eq. Dij-def, eq. A_i), Cholesky ``A_i = L_i L_i^T``,
  MBFs ``A_i phat^(m) = -B_i psi_m`` for ``m`` in ``I_i`` (eq. def-phat-local,
  with ``B_i`` acting as in eq. Bij-contrib) -> interface matrix ``S``.

``S`` is the interface operator of eq. interface-problem-alg written with the
sign of Corollary (Schur complement, eq. k-schur),
``S = Z^T S_lambda Z``, ``S_lambda = -(W + W M Ahat^{-1} B)``, so that
``S[n, m] = -psi_n^T W psi_m + psi_n^T W M phat^(m)`` (using
``Ahat^{-1} B psi_m = -phat^(m)``) and the right-hand side is
``b_n = -psi_n^T W M pbar``.  ``S`` is symmetrised as ``(S + S^T)/2`` before
factoring (it is symmetric in exact arithmetic).

Apply (Algorithm 2, AlgMortarApply): local particular solutions
``A_i pbar_i = r_i`` (eq. def-pbar-local), interface right-hand side, interface
solve, reconstruction ``z = pbar + sum_m eta_m phat^(m)``
(eq. p-decomposition-alg, eq. phat-expansion).

Vectors are kept in original ordering; the subdomain index lists play the role
of the permutation ``P``.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .structure import build_structure

DENSE_S_MAX = 16000


class NotSPDError(ValueError):
    def __init__(self, what, index):
        super().__init__(f"{what} not SPD (index {index})")
        self.what = what
        self.index = index


class AlgMortarCPU:
    """Plain FP64 AlgMortar preconditioner (see module docstring)."""

    def __init__(self, A, part, mortar="interface"):
        self.A = A
        self.st = st = build_structure(A, part, mortar)
        self.n = A.n
        self.m = st.nparts
        As = A.to_scipy().tocsr()
        self.As = As
        part = st.part.astype(np.int64)
        # position of each original index inside its subdomain
        self.loc = np.empty(self.n, dtype=np.int64)
        for i in range(self.m):
            om = st.omega(i)
            self.loc[om] = np.arange(om.size)
        # D = sum_j D_ij: for row k, the sum of a_kl over l outside k's subdomain
        rows = np.repeat(np.arange(self.n), np.diff(A.row_ptr))
        cols = A.col.astype(np.int64)
        outside = part[rows] != part[cols]
        self.d_out = np.bincount(rows[outside], weights=A.val[outside], minlength=self.n)

        # local operators and their Cholesky factors
        self.Ai = []
        self.L = []
        for i in range(self.m):
            om = st.omega(i)
            Aii = As[om][:, om].toarray()
            Ai = Aii - np.diag(self.d_out[om])
            try:
                Li = sla.cholesky(Ai, lower=True)
            except np.linalg.LinAlgError:
                raise NotSPDError("A_i", i) from None
            self.Ai.append(Ai)
            self.L.append(Li)

        # multiscale basis functions, one pair of local pieces per basis function
        self.phat = []
        for nidx in range(st.n_iface):
            i, j = st.iface_ij[nidx]
            pieces = {}
            for s in (int(i), int(j)):
                rhs = -self.B_local(s, nidx)
                pieces[s] = self.local_solve(s, rhs)
            self.phat.append(pieces)
        self.S = self.assemble_S()
        self._factor_S()

    # ---- operators -----------------------------------------------------
    def B_local(self, s, nidx):
        """``B_s psi_n`` on subdomain ``s`` (eq. Bij-contrib, Bi-total-contrib):
        entry ``k`` collects ``2 * a_kl`` over the edges of ``psi_n``'s support
        that are incident to ``k``."""
        st = self.st
        e0, e1 = st.iface_ptr[nidx], st.iface_ptr[nidx + 1]
        out = np.zeros(st.sub_ptr[s + 1] - st.sub_ptr[s])
        for e in range(e0, e1):
            k, l, a = st.edge_k[e], st.edge_l[e], st.edge_a[e]
            if st.part[k] == s:
                out[self.loc[k]] += 2.0 * a
            if st.part[l] == s:
                out[self.loc[l]] += 2.0 * a
        return out

    def local_solve(self, s, rhs):
        """``A_s^{-1} rhs`` with the stored Cholesky factor."""
        return sla.cho_solve((self.L[s], True), rhs)

    def phat_at(self, midx, cells):
        """Values of ``phat^(m)`` at original indices ``cells`` (zero outside
        the two subdomains of ``m``)."""
        out = np.zeros(len(cells))
        parts = self.st.part[cells]
        for s, vals in self.phat[midx].items():
            sel = parts == s
            out[sel] = vals[self.loc[cells[sel]]]
        return out

    def assemble_S(self):
        """``S[n, m] = -delta_nm sum_{e in E_n} a_e
        + sum_{e in E_n} a_e (phat^(m)_k + phat^(m)_l) / 2``, then symmetrised."""
        st = self.st
        NL = st.n_iface
        rows, cols, vals = [], [], []
        for nidx in range(NL):
            e0, e1 = st.iface_ptr[nidx], st.iface_ptr[nidx + 1]
            ks = st.edge_k[e0:e1].astype(np.int64)
            ls = st.edge_l[e0:e1].astype(np.int64)
            a = st.edge_a[e0:e1]
            i, j = st.iface_ij[nidx]
            cand = np.union1d(st.I[i], st.I[j])
            for midx in cand:
                mp = 0.5 * (self.phat_at(midx, ks) + self.phat_at(midx, ls))
                v = float(np.sum(a * mp))
                if midx == nidx:
                    v -= float(np.sum(a))
                rows.append(nidx)
                cols.append(int(midx))
                vals.append(v)
        S = sp.csr_matrix((vals, (rows, cols)), shape=(NL, NL))
        return (0.5 * (S + S.T)).tocsr()

    def _factor_S(self):
        NL = self.st.n_iface
        self._S_dense = None
        self._S_lu = None
        if NL <= DENSE_S_MAX:
            Sd = self.S.toarray()
            try:
                self._S_dense = sla.cho_factor(Sd, lower=True)
            except np.linalg.LinAlgError:
                raise NotSPDError("S", -1) from None
        else:
            self._S_lu = spla.splu(self.S.tocsc())

    def solve_S(self, b):
        if self._S_dense is not None:
            return sla.cho_solve(self._S_dense, b)
        return self._S_lu.solve(b)

    # ---- apply (Algorithm 2) --------------------------------------------
    def local_solves(self, r):
        """``pbar`` with ``A_i pbar_i = r_i`` on every subdomain."""
        st = self.st
        pbar = np.zeros_like(r, dtype=np.float64)
        for i in range(self.m):
            om = st.omega(i)
            pbar[om] = self.local_solve(i, r[om])
        return pbar

    def interface_rhs(self, pbar):
        """``b_n = -sum_{e in E_n} a_e (pbar_k + pbar_l) / 2``."""
        st = self.st
        avg = 0.5 * (pbar[st.edge_k] + pbar[st.edge_l])
        contrib = -(st.edge_a.reshape((-1,) + (1,) * (avg.ndim - 1)) * avg)
        b = np.add.reduceat(contrib, st.iface_ptr[:-1], axis=0) if st.n_edges else \
            np.zeros((0,) + avg.shape[1:])
        return b

    def reconstruct(self, pbar, eta):
        """``z = pbar + sum_m eta_m phat^(m)``."""
        st = self.st
        z = pbar.copy()
        for midx in range(st.n_iface):
            for s, vals in self.phat[midx].items():
                om = st.omega(s)
                if z.ndim == 1:
                    z[om] += eta[midx] * vals
                else:
                    z[om] += vals[:, None] * eta[midx][None, :]
        return z

    def apply(self, r, return_parts=False):
        r = np.asarray(r, dtype=np.float64)
        pbar = self.local_solves(r)
        b = self.interface_rhs(pbar)
        eta = self.solve_S(b)
        z = self.reconstruct(pbar, eta)
        if return_parts:
            return z, dict(pbar=pbar, b=b, eta=eta)
        return z
