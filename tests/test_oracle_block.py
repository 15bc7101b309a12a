"""Pins of the oracle's several-eigenpair variant (Remark after Algorithm 4:
start from p coarse eigenpairs, smooth every vector on each level,
orthogonalise them and take Rayleigh quotients)."""
import math

import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from test_oracle import _path_modes


def _lap(g):
    a = g.to_dense()
    return np.diag(a.sum(1)) - a


def test_coarsest_block_spans_the_lowest_eigenvectors(orc):
    # path P_20: lambda_k = 2 - 2cos(pi k/20), all simple; the block is an
    # orthonormal basis of span(phi_2..phi_{p+1})
    n, p = 20, 3
    V, lams = orc.coarsest_block(G.path(n), p)
    modes, lam = _path_modes(n)
    assert np.allclose(lams, lam[1:p + 1], atol=1e-13)
    assert np.allclose(V.T @ V, np.eye(p), atol=1e-13)
    B = np.array(modes[1:p + 1]).T
    assert np.allclose(B @ (B.T @ V), V, atol=1e-12)  # inside the span
    assert np.allclose(V.sum(0), 0.0, atol=1e-11)


def test_coarsest_block_takes_whole_clusters(orc):
    # 5x5 grid: lambda_2 = lambda_3 (two modes); with p = 1 the start is
    # projected onto the whole 2-dimensional eigenspace
    g = G.grid2d(5, 5)
    V, lams = orc.coarsest_block(g, 1)
    L = _lap(g)
    ev, Q = np.linalg.eigh(L)
    E = Q[:, 1:3]
    assert np.allclose(E @ (E.T @ V), V, atol=1e-12)
    u = np.array([(G.mix64(14120565 ^ 0xD1B54A32D192ED03 ^ 0x9E3779B97F4A7C15 ^ i) >> 11) * 2.0 ** -53
                  for i in range(g.n)]) - 0.5
    pe = E @ (E.T @ u)
    assert np.allclose(V[:, 0], pe / np.linalg.norm(pe), atol=1e-12)


def test_block_pi_orthogonal_iteration_rate(orc):
    # path: columns started at phi_2 + e phi_4 and phi_3 + e phi_4; after k
    # steps of orthogonal iteration the phi_4 component of the block decays
    # like ((g - l4)/(g - l3))^k (subspace iteration)
    n = 24
    g = G.path(n)
    modes, lam = _path_modes(n)
    gv = orc.gershgorin(g)
    eps = 0.2
    V0 = np.stack([modes[1] + eps * modes[3], modes[2] + eps * modes[3]], axis=1)
    r = (gv - lam[3]) / (gv - lam[2])
    for k in (1, 5, 20):
        V, kk, _ = orc.block_pi(g, V0, steps=k)
        assert kk == k
        assert np.allclose(V.T @ V, np.eye(2), atol=1e-13)
        leak = np.linalg.norm(V.T @ modes[3])
        assert leak <= eps * math.sqrt(2) * r ** k * 1.05 + 1e-13


def test_block_pi_exact_eigenvectors_stay(orc):
    n = 30
    g = G.path(n)
    modes, lam = _path_modes(n)
    V0 = np.stack([modes[1], modes[2]], axis=1)
    V, k, mu = orc.block_pi(g, V0, steps=9)
    assert np.allclose(np.abs(V.T @ V0), np.eye(2), atol=1e-12)
    assert abs(mu - 1.0) < 1e-12


def test_cmg_block_ky_fan_and_lapack(orc):
    # Ky Fan: for orthonormal columns orthogonal to 1, the sum of their
    # Rayleigh quotients is at least lambda_2 + ... + lambda_{p+1}; with a
    # tight tolerance the block converges to the eigenpairs (LAPACK)
    g = G.rgg(1500, 10.0, seed=21)
    ev = np.linalg.eigvalsh(_lap(g))
    p = 3
    r = orc.cmg_block(g, p)
    assert r.status == "OK"
    assert np.allclose(r.X.T @ r.X, np.eye(p), atol=1e-12)
    assert np.allclose(r.X.sum(0), 0.0, atol=1e-10)
    assert r.lams.sum() >= ev[1:p + 1].sum() * (1 - 1e-12)
    t = orc.cmg_block(g, p, tol=1e-15, max_iters=200000)
    assert np.allclose(t.lams, ev[1:p + 1], rtol=1e-5)


def test_cmg_block_first_column_tracks_the_fiedler_vector(orc):
    g = G.grid2d(60, 40)  # lambda_2 simple (the long side)
    r = orc.cmg_block(g, 2, tol=1e-12)
    lam2 = 2 - 2 * math.cos(math.pi / 60)
    lam3 = 2 - 2 * math.cos(math.pi / 40)
    assert r.lams[0] == pytest.approx(lam2, rel=1e-3)
    assert r.lams[1] == pytest.approx(lam3, rel=1e-3)


def test_cmg_block_fixed_schedule(orc):
    g = G.grid2d(100, 100)
    r = orc.cmg_block(g, 2, fixed_k0=3, fixed_beta=1.6)
    J = len(r.k) - 1
    assert r.k[:J] == [orc.fixed_steps(3, 1.6, j) for j in range(J)] and r.k[J] == -1
    assert np.allclose(r.X.T @ r.X, np.eye(2), atol=1e-12)


def test_cmg_block_rejects_p_beyond_the_coarsest(orc):
    r = orc.cmg_block(G.path(20), 20)   # dense-only graph of 20 vertices: p <= 19
    assert r.status == "E_ARG"
