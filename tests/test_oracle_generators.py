"""Pins for the seeded input generators (workloads)."""
import math

import numpy as np
import pytest

from workloads import make_config, grf
from workloads.grids import cartesian_faces, distorted_hex_faces
from workloads.fields import layered_log10k
from workloads.tpfa import Faces, assemble


def _check_mmatrix(A, f_has_dirichlet=True):
    S = A.to_scipy()
    assert (S != S.T).nnz == 0, "A must be bitwise symmetric"
    off = S.copy()
    off.setdiag(0)
    off.eliminate_zeros()
    assert off.data.max() < 0, "off-diagonals must be negative"
    rs = S @ np.ones(A.n)
    assert rs.min() > -1e-10 * abs(S.diagonal()).max()
    if f_has_dirichlet:
        assert rs.max() > 0


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_config_is_spd_mmatrix(name):
    P = make_config(name)
    _check_mmatrix(P.A)


def test_config_sizes_match_closed_forms():
    P = make_config("c1")
    # 2-D 5-point: n + 2 * (interior faces)
    assert P.n == 4096 and P.A.nnz == 4096 + 2 * (2 * 63 * 64)
    P = make_config("c2")
    assert P.n == 64 ** 3 and P.A.nnz == 64 ** 3 + 2 * (3 * 63 * 64 * 64)


def test_grf_moments_and_correlation():
    g = grf((256, 256), 8.0, 1.5, 7)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.5) < 1e-12
    # Gaussian covariance: correlation at lag ell is exp(-1/2)
    c = np.mean(g[:, :-8] * g[:, 8:]) / g.var()
    assert abs(c - math.exp(-0.5)) < 0.08
    c2 = np.mean(g[:, :-16] * g[:, 16:]) / g.var()
    assert abs(c2 - math.exp(-2.0)) < 0.08
    # anisotropic lengths act on the right axes
    h = grf((64, 64, 64), (2.0, 16.0, 16.0), 1.0, 3)
    cz = np.mean(h[:-2] * h[2:]) / h.var()
    cx = np.mean(h[:, :, :-2] * h[:, :, 2:]) / h.var()
    assert cz < 0.75 < cx


def test_grf_deterministic():
    assert np.array_equal(grf((16, 16), 4.0, 1.0, 5), grf((16, 16), 4.0, 1.0, 5))
    assert not np.array_equal(grf((16, 16), 4.0, 1.0, 5), grf((16, 16), 4.0, 1.0, 6))


def test_layered_contrast_is_1e6():
    l10 = layered_log10k(64, 64, 64, (16, 16, 2), 1.5, 2)
    assert l10.min() == -3.0 and l10.max() == 3.0


def test_cartesian_factor_is_two():
    f = cartesian_faces(4, 3, 2, [(0, 0, 1.0)])
    assert np.all(f["gk"] == 2.0)
    assert np.all(f["gl"][f["l"] >= 0] == 2.0)
    # unit K, 1-D: interior T = 2*2/(2+2) = 1, Dirichlet t = 2
    A, b = assemble(Faces.from_dict(cartesian_faces(3, 1, 1, [(0, 0, 5.0)])), np.ones(3), 3)
    Ad = A.to_scipy().toarray()
    assert np.array_equal(Ad, np.array([[3.0, -1, 0], [-1, 2, -1], [0, -1, 1]]))
    assert np.array_equal(b, np.array([10.0, 0, 0]))


def test_distorted_hex_zero_jitter_is_cartesian():
    a = distorted_hex_faces(4, 3, 2, 0.0, 1, [(0, 0, 0.0), (2, 1, 1.0)])
    b = cartesian_faces(4, 3, 2, [(0, 0, 0.0), (2, 1, 1.0)])
    for key in ("k", "l", "pD"):
        assert np.array_equal(a[key], b[key])
    assert np.allclose(a["gk"], b["gk"], rtol=0, atol=1e-13)
    assert np.allclose(a["gl"], b["gl"], rtol=0, atol=1e-13)


def test_distorted_hex_positive_and_mmatrix():
    f = Faces.from_dict(distorted_hex_faces(8, 6, 5, 0.3, 11, [(0, 0, 0.0)]))
    assert f.gk.min() > 0
    A, _ = assemble(f, np.exp(np.random.default_rng(0).normal(size=240)), 240)
    _check_mmatrix(A)


def test_cross_pattern_closed_forms():
    """The cross pattern: in every 8^3 tile, cells with at least two of three
    tile coordinates in {3, 4} -- 3 bars of 2x2x8 sharing a 2^3 core, so
    3*32 - 2*8 = 80 cells; kappa in {1, 1e6}; straight channels along x, y
    and z cross the whole grid; the tile is symmetric under a -> 7 - a."""
    from workloads.fields import cross_log_kappa
    lk = cross_log_kappa(24, 16, 8)
    assert set(np.unique(lk)) == {0.0, math.log(1e6)}
    hi = lk > 0
    assert hi.sum() == 80 * (3 * 2 * 1)
    t = hi[:8, :8, :8]
    assert np.array_equal(t, t[::-1, :, :]) and np.array_equal(t, t[:, ::-1, :])
    assert np.array_equal(t, t[:, :, ::-1]) and np.array_equal(t, np.transpose(t, (1, 0, 2)))
    assert hi[3:5, 3:5, :].all() and hi[3:5, :, 3:5].all() and hi[:, 3:5, 3:5].all()
    # a cell off every band is low
    assert not hi[0, 0, 0] and not hi[3, 0, 0]


def test_contrast_sweep_scales_the_contrast():
    """K -> K^theta turns a field of contrast c into one of contrast c^theta."""
    P1 = make_config("c6", nx=16, ny=16, nz=16)
    for th in (0.6, 1.4):
        P = make_config("c6", nx=16, ny=16, nz=16, theta=th)
        K = np.exp(P.logK)
        assert math.isclose(K.max() / K.min(), 1e6 ** th, rel_tol=1e-12)
        assert np.allclose(P.logK, th * P1.logK, rtol=0, atol=0)
    Pl1 = make_config("c2", nx=16, ny=16, nz=16)
    Pl = make_config("c2", nx=16, ny=16, nz=16, theta=1.4)
    c1 = np.exp(Pl1.logK).max() / np.exp(Pl1.logK).min()
    c = np.exp(Pl.logK).max() / np.exp(Pl.logK).min()
    assert math.isclose(c, c1 ** 1.4, rel_tol=1e-9)


def test_cross_config_is_spd_mmatrix():
    P = make_config("c6", nx=16, ny=16, nz=16)
    _check_mmatrix(P.A)
    assert P.partition == ("blocks", (8, 8, 8)) and P.tol == 1e-8
