"""Pins for the oracle's muscles: special cases that reduce to LAPACK routines."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle.primitives import left_solve_upper_t, right_solve_upper


def _spd(s, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
    lam = np.logspace(0, np.log10(cond), s)
    M = (Q * lam) @ Q.T
    return 0.5 * (M + M.T)


@pytest.mark.parametrize("s", [1, 2, 4, 8, 16, 32])
def test_chol_flag_matches_lapack_potrf(s):
    Om = _spd(s, 100 + s)
    R, ok = oracle.chol_flag(Om)
    assert ok
    # LAPACK potrf (upper) is the reference factorization
    Rl, info = sla.lapack.dpotrf(Om, lower=0, clean=1)
    assert info == 0
    assert np.linalg.norm(R - Rl) <= 1e-13 * np.linalg.norm(Rl)
    assert np.allclose(np.tril(R, -1), 0.0)


def test_chol_flag_reads_upper_triangle_only():
    Om = _spd(6, 7)
    junk = Om.copy()
    junk[np.tril_indices(6, -1)] = 123.0     # garbage below the diagonal
    R1, ok1 = oracle.chol_flag(Om)
    R2, ok2 = oracle.chol_flag(junk)
    assert ok1 and ok2 and np.array_equal(R1, R2)


@pytest.mark.parametrize("seed", range(6))
def test_chol_flag_agrees_with_potrf_info_on_indefinite(seed):
    rng = np.random.default_rng(seed)
    s = 5
    Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
    lam = np.array([3.0, 2.0, 1.0, 0.5, -0.1 * (seed + 1)])
    Om = (Q * lam) @ Q.T
    Om = 0.5 * (Om + Om.T)
    _, ok = oracle.chol_flag(Om)
    _, info = sla.lapack.dpotrf(Om, lower=0)
    assert (not ok) and info > 0


@pytest.mark.parametrize("bad", ["zero", "nan", "inf", "negdiag"])
def test_chol_flag_special_cases(bad):
    Om = np.eye(3)
    if bad == "zero":
        Om = np.zeros((3, 3))
    elif bad == "nan":
        Om[1, 1] = np.nan
    elif bad == "inf":
        Om[2, 2] = np.inf
    else:
        Om[0, 0] = -1.0
    assert not oracle.chol_flag(Om)[1]


@pytest.mark.parametrize("s", [1, 3, 8])
def test_cholqr_matches_householder_qr(s):
    rng = np.random.default_rng(s)
    X = rng.standard_normal((200, s)) @ np.diag(np.logspace(0, 2, s))
    Q, R, ok = oracle.cholqr(X)
    assert ok
    Qh, Rh = np.linalg.qr(X)
    d = np.sign(np.diag(Rh))
    Qh, Rh = Qh * d, d[:, None] * Rh
    assert np.linalg.norm(R - Rh) <= 1e-12 * np.linalg.norm(Rh)
    assert np.linalg.norm(Q - Qh) <= 1e-11


def test_cholqr_flags_rank_deficient_block():
    """A zero column gives an exactly zero pivot.  (A column that is only
    numerically dependent may leave a tiny positive pivot: CholQR flags only
    a numerically non-positive-definite Gram matrix.)"""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, 3))
    X[:, 2] = 0.0
    assert not oracle.cholqr(X)[2]


@pytest.mark.parametrize("s", [1, 4, 16])
def test_houseqr_is_a_positive_diagonal_qr(s):
    rng = np.random.default_rng(10 + s)
    X = rng.standard_normal((300, s))
    Q, R, ok = oracle.houseqr(X)
    assert ok
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert np.linalg.norm(Q.T @ Q - np.eye(s)) <= 1e-14 * s
    assert np.linalg.norm(Q @ R - X) <= 1e-14 * np.linalg.norm(X) * s


def test_triangular_helpers_against_explicit_inverse():
    R = np.triu(_spd(5, 1)) + 5 * np.eye(5)
    X = np.random.default_rng(0).standard_normal((7, 5))
    assert np.allclose(right_solve_upper(X, R), X @ np.linalg.inv(R), rtol=1e-13, atol=1e-14)
    Y = np.random.default_rng(1).standard_normal((5, 3))
    assert np.allclose(left_solve_upper_t(R, Y), np.linalg.inv(R).T @ Y, rtol=1e-13, atol=1e-14)


def test_intra_ortho_t_factor_is_identity():
    X = np.random.default_rng(2).standard_normal((40, 4))
    for musc in ("cholqr", "houseqr"):
        Q, R, T, ok = oracle.intra_ortho(X, musc)
        assert ok and np.array_equal(T, np.eye(4))
    with pytest.raises(ValueError):
        oracle.intra_ortho(X, "tsqr")


@pytest.mark.parametrize("muscle", ["mgs_svl", "mgs_lts"])
def test_mgs_lowsync_muscles(muscle):
    """Column-wise MGS-SVL / MGS-LTS (Sec. 5 muscles): X = Q R with R upper
    triangular, positive diagonal, equal to the unique Householder R with
    diag(R) > 0 on a well-conditioned block; T is unit upper triangular and
    encodes the computed loss of orthogonality: SVL T^{-1} = I + triu(Q^T Q, 1),
    LTS T = I + triu(Q^T Q, 1) (the Schreiber-Van Loan and lower-triangular-
    solve representations)."""
    from oracle.primitives import houseqr, intra_ortho
    rng = np.random.default_rng(3)
    X = rng.standard_normal((400, 6))
    # a few nearly dependent columns make the loss of orthogonality visible
    X[:, 4] = X[:, 1] + 1e-6 * rng.standard_normal(400)
    Q, R, T, ok = intra_ortho(X, muscle)
    assert ok
    assert np.linalg.norm(Q @ R - X) <= 1e-13 * np.linalg.norm(X)
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) > 0)
    U = np.triu(Q.T @ Q, 1)
    assert np.allclose(np.tril(T, -1), 0.0) and np.allclose(np.diag(T), 1.0)
    if muscle == "mgs_svl":
        assert np.linalg.norm(np.linalg.inv(T) - (np.eye(6) + U)) <= 1e-12
    else:
        assert np.linalg.norm(T - (np.eye(6) + U)) <= 1e-12
    # well-conditioned block: the unique QR (Householder with diag(R) > 0)
    Y = rng.standard_normal((300, 5))
    Qm, Rm, Tm, okm = intra_ortho(Y, muscle)
    Qh, Rh, okh = houseqr(Y)
    assert okm and okh
    assert np.linalg.norm(Rm - Rh) <= 1e-12 * np.linalg.norm(Rh)
    assert np.linalg.norm(Qm - Qh) <= 1e-12
    assert np.linalg.norm(Tm - np.eye(5)) <= 1e-13


def test_mgs_muscle_flags_a_zero_column():
    """A zero column leaves w = 0 exactly: w^T w is not positive, so the
    muscle raises the flag (as CholQR does for the same block)."""
    from oracle.primitives import intra_ortho
    X = np.zeros((50, 3))
    X[:, 0] = 1.0
    X[:, 1] = np.arange(50.0)
    for muscle in ("mgs_svl", "mgs_lts"):
        _, _, _, ok = intra_ortho(X, muscle)
        assert not ok
