"""Adjoint gradient of a least-squares loss with respect to ``theta = ln K``.

No paper analogue (the paper has no adjoint); written from the calculus of the
TPFA residual ``R(p, theta) = A(theta) p - f(theta) = 0``:

* loss ``J = 1/2 sum_{c in obs} (p_c - pobs_c)^2``;
* adjoint ``A^T lambda = dJ/dp`` (``A`` symmetric, so the same solver applies);
* ``dJ/dtheta = -lambda^T (dA/dtheta p - df/dtheta)``, i.e. for each cell ``c``

      dJ/dtheta_c = - sum_{interior faces f = (k, l) touching c}
                        dT_f/dtheta_c * (lambda_k - lambda_l) * (p_k - p_l)
                    - sum_{Dirichlet faces of c} t_c * lambda_c * (p_c - pD)

  with ``T = t_k t_l / (t_k + t_l)``, ``t_c = K_c g_c`` and hence
  ``dT/dtheta_k = T t_l / (t_k + t_l)``, ``dT/dtheta_l = T t_k / (t_k + t_l)``,
  ``dt_c/dtheta_c = t_c``.
"""
import numpy as np


def loss(p, obs, pobs):
    d = p[obs] - pobs
    return 0.5 * float(d @ d)


def dloss_dp(p, obs, pobs):
    g = np.zeros_like(p)
    g[obs] = p[obs] - pobs
    return g


def tpfa_values(faces, logK):
    """Half-transmissibilities and interior transmissibilities for ``ln K``."""
    K = np.exp(logK)
    tk = K[faces.k] * faces.gk
    interior = faces.l >= 0
    tl = np.zeros_like(tk)
    tl[interior] = K[faces.l[interior]] * faces.gl[interior]
    T = np.zeros_like(tk)
    T[interior] = tk[interior] * tl[interior] / (tk[interior] + tl[interior])
    return tk, tl, T


def gradient(faces, logK, p, lam):
    """``dJ/dtheta`` from state ``p`` and adjoint ``lam`` (formula above)."""
    n = logK.size
    tk, tl, T = tpfa_values(faces, logK)
    interior = faces.l >= 0
    k = faces.k[interior]
    l = faces.l[interior]
    tki, tli, Ti = tk[interior], tl[interior], T[interior]
    flux = (lam[k] - lam[l]) * (p[k] - p[l])
    dT_dk = Ti * tli / (tki + tli)
    dT_dl = Ti * tki / (tki + tli)
    g = -(np.bincount(k, weights=dT_dk * flux, minlength=n)
          + np.bincount(l, weights=dT_dl * flux, minlength=n))
    bnd = ~interior
    kb = faces.k[bnd]
    g -= np.bincount(kb, weights=tk[bnd] * lam[kb] * (p[kb] - faces.pD[bnd]), minlength=n)
    return g
