"""Dense matrices of the paper's operators, for identities on small cases.

Built straight from the definitions in Sec. 3.2 (incidence ``C_ij``,
restrictions, weight ``W`` eq. global-W, traces ``L``/``U`` eq. L-operator,
U-operator, average ``M`` eq. avg-operator, coupling ``B`` eq. Bij-matrix-form
and def-B), Sec. 3.3 (``Ahat``), Sec. 4 (``Q`` eq. Q-def) and Sec. 5 (the
reduced preconditioner eq. m-reduced-p and the spectral bound eq. k-lambda).
All matrices are in original ordering; ``Z`` spans the mortar space.
"""
import numpy as np
import scipy.linalg as sla


def operators(pre):
    """Dense ``W, L, U, M, B, Z, Ahat`` for an :class:`AlgMortarCPU` ``pre``."""
    st = pre.st
    n, ne, NL = st.n, st.n_edges, st.n_iface
    W = np.diag(st.edge_a)
    L = np.zeros((ne, n))
    U = np.zeros((ne, n))
    L[np.arange(ne), st.edge_k] = 1.0
    U[np.arange(ne), st.edge_l] = 1.0
    M = 0.5 * (L + U)
    # B = stacked B_i, (B mu)_k = 2 sum_{l:(k,l) in E} a_kl mu(k,l), both endpoints
    B = np.zeros((n, ne))
    B[st.edge_k, np.arange(ne)] += 2.0 * st.edge_a
    B[st.edge_l, np.arange(ne)] += 2.0 * st.edge_a
    Z = np.zeros((ne, NL))
    for nidx in range(NL):
        Z[st.iface_ptr[nidx]:st.iface_ptr[nidx + 1], nidx] = 1.0
    Ahat = np.zeros((n, n))
    for i in range(pre.m):
        om = st.omega(i)
        Ahat[np.ix_(om, om)] = pre.Ai[i]
    return dict(W=W, L=L, U=U, M=M, B=B, Z=Z, Ahat=Ahat)


def reduced_preconditioner(ops):
    """``Mcal = Ahat + 4 M^T W Z (Z^T W Z)^{-1} Z^T W M`` (eq. m-reduced-p)."""
    W, M, Z, Ahat = ops["W"], ops["M"], ops["Z"], ops["Ahat"]
    ZWZ = Z.T @ W @ Z
    return Ahat + 4.0 * M.T @ W @ Z @ np.linalg.solve(ZWZ, Z.T @ W @ M)


def Q_matrix(ops):
    """Symmetric saddle form ``Q`` of Proposition (eq. Q-def)."""
    W, M, Z, Ahat = ops["W"], ops["M"], ops["Z"], ops["Ahat"]
    top = np.hstack([0.25 * Ahat, M.T @ W @ Z])
    bot = np.hstack([Z.T @ W @ M, -Z.T @ W @ Z])
    return np.vstack([top, bot])


def K_lambda(ops, Adense):
    """``K_Lambda = max_p 4 ||(I - Pi) M p||_{-W}^2 / ||p||_A^2`` (eq. k-lambda)
    as the largest generalized eigenvalue."""
    W, M, Z = ops["W"], ops["M"], ops["Z"]
    Pi = Z @ np.linalg.solve(Z.T @ W @ Z, Z.T @ W)
    R = (np.eye(W.shape[0]) - Pi) @ M
    num = 4.0 * R.T @ (-W) @ R
    num = 0.5 * (num + num.T)
    return float(sla.eigh(num, Adense, eigvals_only=True)[-1])


def to_dense(A):
    return A.to_scipy().toarray()
