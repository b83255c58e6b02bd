"""The band factorisation and solve kernels of Steps 1 and 3 on their own,
through lp_band_factor_solve: solutions against LAPACK's banded solver, the
pivot and growth monitor against a plain elimination, and the monitor's
flag on a small pivot and on a large growth factor."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2311_05170_amd import lib

pytestmark = pytest.mark.gpu


def band_of(A, bw):
    """(n, n) dense -> (n, 2 bw + 1) band storage, entry (i, j) at [j, i - j + bw]."""
    n = A.shape[0]
    B = np.zeros((n, 2 * bw + 1))
    for d in range(-bw, bw + 1):
        j = np.arange(max(0, -d), min(n, n - d))
        B[j, d + bw] = A[j + d, j]
    return B


def random_band(rng, n, bw, dominant=True):
    A = np.zeros((n, n))
    for d in range(-bw, bw + 1):
        idx = np.arange(max(0, -d), min(n, n - d))
        A[idx + d, idx] = rng.uniform(-1, 1, len(idx))
    if dominant:
        A[np.arange(n), np.arange(n)] = 2 * bw + 3 + rng.uniform(0, 1, n)
    return A


def lapack_solve(A, b, bw):
    n = A.shape[0]
    ab = np.zeros((2 * bw + 1, n))
    for d in range(-bw, bw + 1):
        j = np.arange(max(0, -d), min(n, n - d))
        ab[bw + d, j] = A[j + d, j]
    return sla.solve_banded((bw, bw), ab, b)


def plain_elimination(A):
    """Gaussian elimination without pivoting: (growth max|u_ij| / max|a_ij|,
    smallest |u_kk| / max|a_ij|)."""
    U = A.astype(np.float64).copy()
    n = U.shape[0]
    for k in range(n - 1):
        U[k + 1:, k + 1:] -= np.outer(U[k + 1:, k] / U[k, k], U[k, k + 1:])
        U[k + 1:, k] = 0.0
    amax = np.abs(A).max()
    return np.abs(np.triu(U)).max() / amax, np.abs(np.diag(U)).min() / amax


CASES = [(1, 0), (13, 3), (37, 5), (300, 40), (517, 64), (700, 95), (1000, 128), (1203, 159)]


@pytest.mark.parametrize("variant", [9, 8, 0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_band_solve_matches_lapack(variant, precision):
    """Three systems per case, ragged sizes in every window class; FP64
    factors to 1e-12, FP32 factors (no refinement) to 2e-6, relative."""
    rng = np.random.default_rng(11)
    for n, bw in CASES:
        As = [random_band(rng, n, bw) for _ in range(3)]
        band = np.stack([band_of(A, bw) for A in As])
        rhs = rng.standard_normal((3, n))
        x, flags, growth, pivot = lib.band_factor_solve(band, rhs, precision, variant)
        tol = 1e-12 if precision == "fp64" else 2e-6
        for s in range(3):
            ref = lapack_solve(As[s], rhs[s], bw)
            err = np.abs(x[s] - ref).max() / np.abs(ref).max()
            assert err < tol, (n, bw, s, err)
        assert flags == 0, (n, bw, flags)


@pytest.mark.parametrize("variant", [9, 0])
def test_band_monitor_values(variant):
    """Growth factor and smallest relative pivot as a plain elimination finds
    them (diagonally dominant: growth at most 2), to float rounding."""
    rng = np.random.default_rng(12)
    n, bw = 240, 30
    As = [random_band(rng, n, bw) for _ in range(2)]
    As[1][np.arange(n), np.arange(n)] *= 0.6
    band = np.stack([band_of(A, bw) for A in As])
    ref = [plain_elimination(A) for A in As]
    for precision in ("fp64", "mixed"):
        _, flags, growth, pivot = lib.band_factor_solve(band, np.ones((2, n)), precision, variant)
        assert flags == 0
        tol = 1e-5 if precision == "fp64" else 1e-4
        assert abs(growth - max(r[0] for r in ref)) < tol * growth, (growth, ref)
        assert abs(pivot - min(r[1] for r in ref)) < tol * pivot, (pivot, ref)
        assert growth <= 2.0


@pytest.mark.parametrize("variant", [9, 8, 0])
def test_small_pivot_raises_flag(variant):
    """A pivot that only elimination makes small (rows 40-41 hold
    [[1, 1], [1, 1 + d]]: the second pivot is d, against a largest entry of
    16) raises bit 2 below one rounding unit of the largest entry (2^-23 in
    FP32, 2^-52 in FP64) and not above it."""
    n, bw = 120, 12
    rng = np.random.default_rng(13)
    base = random_band(rng, n, bw)
    base /= np.abs(base).max()
    base[0, 0] = 16.0
    # powers of two: 1 + d is exact in the factor's precision; d / 16 is the
    # relative pivot
    for precision, d_small, d_ok in (("mixed", 2.0 ** -20, 2.0 ** -14), ("fp64", 2.0 ** -50, 2.0 ** -40)):
        got = []
        for d in (d_small, d_ok):
            A = base.copy()
            A[40:42, :] = 0.0
            A[:, 40:42] = 0.0
            A[40, 40], A[40, 41], A[41, 40], A[41, 41] = 1.0, 1.0, 1.0, 1.0 + d
            _, flags, growth, pivot = lib.band_factor_solve(band_of(A, bw)[None], np.ones((1, n)), precision, variant)
            got.append((flags, pivot))
            assert abs(pivot - d / 16) < 0.05 * d / 16, (precision, d, pivot)
        assert got[0][0] & 4, (precision, got)
        assert not (got[1][0] & 4), (precision, got)


def test_large_growth_raises_flag():
    """Wilkinson's matrix (unit diagonal, -1 below it, last column of ones)
    has growth 2^(n-1) without pivoting and no small pivot: n = 18 passes in
    FP32 (2^17 > 2^16 flags), n = 16 (2^15) does not."""
    for n, flagged in ((18, True), (16, False)):
        A = np.eye(n) - np.tril(np.ones((n, n)), -1)
        A[:, -1] = 1.0
        bw = n - 1
        for variant in (9, 0):
            _, flags, growth, pivot = lib.band_factor_solve(band_of(A, bw)[None], np.ones((1, n)), "mixed", variant)
            assert abs(growth - 2.0 ** (n - 1)) < 1e-3 * growth, (n, growth)
            assert bool(flags & 4) == flagged, (n, variant, flags)
