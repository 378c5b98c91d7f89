"""Pins of the oracle's inner iterations, colouring and scaling (CPU only).

Each check compares the oracle with something other than itself: the matrix form of the
inner iterations given in Sec. 3.1/3.2 of the paper (C<l> = sum_{i<l} H^i M^-1 with the
splitting A A^T = M - N), the textbook SOR/SSOR splittings, Richardson's closed form,
eigenvalues from LAPACK, and the defining property of the greedy colouring.
"""
import numpy as np
import pytest

import oracle
from paper_1604_07491_amd import synth


def _rand_csr(m, n, density, seed, dup=0):
    rng = np.random.default_rng(seed)
    while True:
        A = rng.standard_normal((m, n)) * (rng.random((m, n)) < density)
        if np.all(np.abs(A).sum(1) > 0) and np.all(np.abs(A).sum(0) > 0):
            break
    if dup:
        A = np.concatenate([A, A[:dup]], 0)
    return synth.from_dense(A, np.zeros(A.shape[0]), np.zeros(n)), A


# ---------------------------------------------------------------------------- colouring
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_colouring_is_valid_and_greedy(seed):
    lp, A = _rand_csr(40, 60, 0.08, seed)
    col, perm, nc = oracle.colour(lp)
    nzs = [set(np.nonzero(A[i])[0]) for i in range(lp.m)]
    # rows of one colour share no column
    for i in range(lp.m):
        for k in range(i):
            if col[i] == col[k]:
                assert not (nzs[i] & nzs[k])
    # greedy: every smaller colour is used by an earlier conflicting row
    for i in range(lp.m):
        used = {col[k] for k in range(i) if nzs[i] & nzs[k]}
        assert col[i] == min(set(range(lp.m + 1)) - used)
    # colour-major order, ascending rows inside a colour
    assert sorted(perm.tolist()) == list(range(lp.m))
    keys = [(col[r], r) for r in perm]
    assert keys == sorted(keys)
    assert nc == col.max() + 1


def test_colouring_special_cases():
    # a dense matrix is a complete conflict graph: colour = row (natural order)
    lp, _ = _rand_csr(12, 20, 1.0, 5)
    col, perm, nc = oracle.colour(lp)
    assert nc == 12 and np.array_equal(col, np.arange(12)) and np.array_equal(perm, np.arange(12))
    # a transportation matrix is bipartite: sources get colour 0 and sinks colour 1
    t = synth.transport_lp(7, 5, seed=3)
    col, perm, nc = oracle.colour(t)
    assert nc == 2 and np.all(col[:7] == 0) and np.all(col[7:] == 1)


# ---------------------------------------------------------------------------- NE-SOR
def _sor_closed_form(G, g, omega, ell, rn2):
    """p = C<l> g with C<l> = sum_{i<l} H^i M^-1, M = diag(G)/omega + strict lower(G)."""
    Dg = np.diag(rn2)
    M = Dg / omega + np.tril(G, -1)
    Minv = np.linalg.inv(M)
    H = np.eye(len(g)) - Minv @ G
    C = sum(np.linalg.matrix_power(H, i) for i in range(ell)) @ Minv
    return C @ g


@pytest.mark.parametrize("omega,ell,seed", [(1.0, 1, 0), (1.0, 2, 1), (1.3, 3, 2), (0.7, 2, 3)])
def test_nesor_equals_sor_on_normal_equations(omega, ell, seed):
    """NE-SOR in a given row order is SOR on A A^T p = g in that order (Sec. 3.4 /
    Bjorck-Elfving), i.e. p = C<l> g with the SOR splitting; and z = A^T p."""
    lp, A = _rand_csr(15, 25, 0.3, seed, dup=2)
    rng = np.random.default_rng(seed + 10)
    g = rng.standard_normal(lp.m)
    _, perm, _ = oracle.colour(lp)
    rn2 = (A * A).sum(1)
    z, p = oracle.nesor(lp, g, omega=omega, ell=ell, perm=perm, rn2=rn2)
    Ap = A[perm]
    G = Ap @ Ap.T
    p_ref = np.empty(lp.m)
    p_ref[perm] = _sor_closed_form(G, g[perm], omega, ell, rn2[perm])
    np.testing.assert_allclose(p, p_ref, rtol=1e-10, atol=1e-10 * np.abs(p_ref).max())
    np.testing.assert_allclose(z, A.T @ p, rtol=1e-10, atol=1e-12 * np.abs(z).max())


def test_nesor_unit_rows_matches_division_form():
    """With unit row norms the division by ||alpha_i||^2 is dropped (Sec. 3.5)."""
    lp, A = _rand_csr(12, 20, 0.4, 7)
    rho, ah = oracle.scale(lp)
    lph = synth.LP(lp.m, lp.n, lp.row_ptr, lp.col_idx, ah, lp.b, lp.c)
    g = np.random.default_rng(1).standard_normal(lp.m)
    z1, p1 = oracle.nesor(lph, g, perm=np.arange(lp.m, dtype=np.int32))
    z2, p2 = oracle.nesor(lph, g, perm=np.arange(lp.m, dtype=np.int32), rn2=np.ones(lp.m))
    assert np.array_equal(z1, z2) and np.array_equal(p1, p2)
    Ah = lph.to_dense()
    np.testing.assert_allclose(p1, _sor_closed_form(Ah @ Ah.T, g, 1.0, 2, np.ones(lp.m)), rtol=1e-10)


def test_colour_order_sweep_is_a_sequential_sweep():
    """Rows of one colour share no column, so sweeping the colours in any order of their
    rows gives the same result: a sweep in colour order equals one where the rows inside
    every colour are visited backwards (bitwise, each row dot is the same sum)."""
    lp = synth.sparse_lp(60, 150, 4, 2, seed=9)
    col, perm, nc = oracle.colour(lp)
    g = np.random.default_rng(2).standard_normal(lp.m)
    z1, p1 = oracle.nesor(lp, g, perm=perm, rn2=np.ones(lp.m))
    perm2 = np.concatenate([perm[col[perm] == c][::-1] for c in range(nc)]).astype(np.int32)
    z2, p2 = oracle.nesor(lp, g, perm=perm2, rn2=np.ones(lp.m))
    assert np.array_equal(p1, p2) and np.array_equal(z1, z2)


# ---------------------------------------------------------------------------- NE-SSOR
@pytest.mark.parametrize("omega,ell", [(1.0, 1), (1.2, 3), (0.8, 2)])
def test_nessor_equals_ssor_splitting(omega, ell):
    """NE-SSOR (Sec. 3.3) is SSOR on A A^T p = g: M = w/(2-w) (D/w + L) D^-1 (D/w + U);
    for odd l and w in (0, 2) C<l> is symmetric positive definite."""
    lp, A = _rand_csr(14, 22, 0.35, 11, dup=1)
    perm = np.arange(lp.m, dtype=np.int32)
    rn2 = (A * A).sum(1)
    G = A @ A.T
    Dg = np.diag(rn2)
    M = omega / (2 - omega) * (Dg / omega + np.tril(G, -1)) @ np.linalg.inv(Dg) @ (Dg / omega + np.triu(G, 1))
    Minv = np.linalg.inv(M)
    H = np.eye(lp.m) - Minv @ G
    Cl = sum(np.linalg.matrix_power(H, i) for i in range(ell)) @ Minv
    rng = np.random.default_rng(3)
    g = rng.standard_normal(lp.m)
    z, p = oracle.nesor(lp, g, omega=omega, ell=ell, perm=perm, rn2=rn2, ssor=True)
    np.testing.assert_allclose(p, Cl @ g, rtol=1e-9, atol=1e-10 * np.abs(p).max())
    np.testing.assert_allclose(z, A.T @ p, rtol=1e-9, atol=1e-11 * np.abs(z).max())
    if ell % 2 == 1:
        # C<l> from the oracle itself, column by column
        Cor = np.stack([oracle.nesor(lp, e, omega=omega, ell=ell, perm=perm, rn2=rn2, ssor=True)[1]
                        for e in np.eye(lp.m)], 1)
        np.testing.assert_allclose(Cor, Cor.T, atol=1e-9 * np.abs(Cor).max())
        assert np.linalg.eigvalsh((Cor + Cor.T) / 2).min() > 0


# ---------------------------------------------------------------------------- Cimmino
def test_cimmino_is_richardson():
    """Cimmino sweeps are Richardson steps on A A^T p = g: p = sum_{i<l} (I - wG)^i w g."""
    lp, A = _rand_csr(10, 30, 0.3, 4)
    G = A @ A.T
    lam_max = np.linalg.eigvalsh(G).max()
    lam = oracle.power_lambda(lp, 20)
    assert lam <= lam_max * (1 + 1e-12) and lam >= 0.5 * lam_max
    w = 1.0 / lam
    g = np.random.default_rng(0).standard_normal(lp.m)
    for ell in (1, 2, 4):
        z, p = oracle.cimmino(lp, g, w, ell)
        R = np.eye(lp.m) - w * G
        p_ref = sum(np.linalg.matrix_power(R, i) for i in range(ell)) @ (w * g)
        np.testing.assert_allclose(p, p_ref, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(z, A.T @ p, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------- scaling
def test_scaling_unit_rows():
    """A_hat = diag(rho)^-1 A D has unit rows (Sec. 3.5) and rho_i = ||row i of A D||."""
    lp, A = _rand_csr(9, 17, 0.5, 8)
    d = np.random.default_rng(5).uniform(0.1, 3.0, lp.n)
    rho, ah = oracle.scale(lp, d)
    AD = A * d[None, :]
    np.testing.assert_allclose(rho, np.linalg.norm(AD, axis=1), rtol=1e-14)
    Ah = synth.LP(lp.m, lp.n, lp.row_ptr, lp.col_idx, ah, lp.b, lp.c).to_dense()
    np.testing.assert_allclose(Ah, AD / rho[:, None], rtol=1e-14, atol=0)
    np.testing.assert_allclose(np.linalg.norm(Ah, axis=1), 1.0, rtol=1e-14)


def test_csr_products_match_dense():
    lp, A = _rand_csr(11, 19, 0.4, 12)
    x = np.random.default_rng(1).standard_normal(lp.n)
    y = np.random.default_rng(2).standard_normal(lp.m)
    np.testing.assert_allclose(oracle.csr_mv(lp, x), A @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.csr_tmv(lp, y), A.T @ y, rtol=1e-13, atol=1e-13)
