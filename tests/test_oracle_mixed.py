"""Pins of the oracle's mixed-precision steps: the split overlap and product of
CholGS (Sec. 3.4, eq. overlapmixedprec and the product after it) and the
split projected Hamiltonian of Rayleigh-Ritz (Sec. 3.5, eq.
partialDiagMixedPrec1 and its limit eq. partialDiagLim2).

What fixes them, independently of the functions under test:
* exactly rounded sums (``math.fsum``) of the products: of the FP64 inputs
  for the blocks the paper keeps in FP64 (error at FP64 level), and of the
  inputs rounded to FP32 -- whose pairwise products are exact in FP64 -- for
  the blocks it moves to FP32, where the error must lie inside the classical
  FP32 accumulation bound gamma_n(u32) sum |x y| and far above anything an
  FP64 accumulation (or FP64 inputs) could leave;
* small-integer data, for which FP32 arithmetic is exact in any order, so the
  split results are bit-equal to the exact integer products (a dropped,
  transposed or mis-indexed block fails);
* the paper's limit: on exact eigenvectors the coupling blocks vanish and the
  fractionally occupied Ritz values keep FP64 accuracy.
"""
import math

import numpy as np
import pytest

from oracle import chfsi, density, fem

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _fsum_dot(x, y):
    return math.fsum((x * y).tolist())


def _gamma32(n):
    return n * U32 / (1.0 - n * U32)


def _check_split_product(A, B, got, fp64_mask):
    """got ~ A^T B: entries where fp64_mask holds at FP64 level, the others at
    FP32 level (inputs rounded, FP32 sums) -- returns the largest FP32-block
    deviation from the FP32-input exact sum and from the FP64 sum, each
    relative to the FP64 rounding scale n u64 sum |a b|."""
    n = A.shape[0]
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    worst_r, worst_64 = 0.0, 0.0
    for i in range(A.shape[1]):
        for j in range(B.shape[1]):
            if fp64_mask[i, j]:
                ref = _fsum_dot(A[:, i], B[:, j])
                bound = (n + 2) * U64 * float(np.abs(A[:, i]) @ np.abs(B[:, j]))
                assert abs(got[i, j] - ref) <= bound, (i, j, got[i, j] - ref, bound)
            else:
                ref_r = _fsum_dot(A32[:, i], B32[:, j])         # exact products, one rounding
                mag = float(np.abs(A32[:, i]) @ np.abs(B32[:, j]))
                assert abs(got[i, j] - ref_r) <= _gamma32(n) * mag + U64 * abs(ref_r), (i, j)
                floor = n * U64 * mag
                ref64 = _fsum_dot(A[:, i], B[:, j])
                worst_r = max(worst_r, abs(got[i, j] - ref_r) / floor)
                worst_64 = max(worst_64, abs(got[i, j] - ref64) / floor)
    return worst_r, worst_64


def test_overlap_mixed_fp64_diagonal_blocks_fp32_elsewhere():
    rng = np.random.default_rng(901)
    X = rng.standard_normal((2000, 40))
    bv = 16
    S = chfsi.overlap_mixed(X, bv)
    blk = np.arange(40) // bv
    diag = blk[:, None] == blk[None, :]
    worst_r, worst_64 = _check_split_product(X, X, S, diag)
    # FP32 accumulation really ran off the diagonal blocks (an FP64 sum of the
    # rounded inputs would sit within 1 of this scale), and the inputs really
    # were rounded (an FP64 off-diagonal block would too)
    assert worst_r > 100.0 and worst_64 > 100.0, (worst_r, worst_64)
    # the diagonal blocks are the FP64 Gram's own entries
    G = X.T @ X
    assert np.array_equal(S[diag], G[diag])


def test_rmul_mixed_fp64_diagonal_blocks_fp32_elsewhere():
    rng = np.random.default_rng(902)
    X = rng.standard_normal((1500, 36))
    U = np.triu(rng.standard_normal((36, 36)))
    bv = 12
    blk = np.arange(36) // bv
    diag = blk[:, None] == blk[None, :]
    got = chfsi.rmul_mixed(X, U, bv)
    X32 = X.astype(np.float32).astype(np.float64)
    U32a = U.astype(np.float32).astype(np.float64)
    worst = 0.0
    for r in range(0, 1500, 37):
        for j in range(36):
            d = diag[:, j]
            ref_d = math.fsum((X[r, d] * U[d, j]).tolist())
            ref_o = math.fsum((X32[r, ~d] * U32a[~d, j]).tolist())
            mag_o = float(np.abs(X32[r, ~d]) @ np.abs(U32a[~d, j]))
            mag_d = float(np.abs(X[r, d]) @ np.abs(U[d, j]))
            err = abs(got[r, j] - (ref_d + ref_o))
            assert err <= _gamma32(36) * mag_o + 40 * U64 * (mag_d + mag_o), (r, j, err)
            ref64 = math.fsum((X[r, :] * U[:, j]).tolist())
            if mag_o > 0:
                worst = max(worst, abs(got[r, j] - ref64) / (36 * U64 * (mag_o + mag_d)))
    assert worst > 100.0, worst            # the off-diagonal part ran in FP32


def test_mixed_steps_bit_exact_where_fp32_is_exact():
    """Small integers: every FP32 product and partial sum is an integer below
    2^24, so the split results equal the exact integer products bit for bit."""
    rng = np.random.default_rng(903)
    X = rng.integers(-8, 9, size=(500, 48)).astype(np.float64)
    U = np.triu(rng.integers(-4, 5, size=(48, 48))).astype(np.float64)
    Xi = X.astype(np.int64)
    assert np.array_equal(chfsi.overlap_mixed(X, 16), (Xi.T @ Xi).astype(np.float64))
    assert np.array_equal(chfsi.rmul_mixed(X, U, 16), (Xi @ U.astype(np.int64)).astype(np.float64))
    HX = rng.integers(-8, 9, size=(500, 48)).astype(np.float64)
    assert np.array_equal(density.projected_split(X, HX, 30), (Xi.T @ HX.astype(np.int64)).astype(np.float64))


def test_cholgs_mixed_equals_fp64_when_off_diagonal_blocks_vanish():
    """Blocks of columns with disjoint row supports: S and L^-T are block
    diagonal (the off-diagonal FP32 products are exact zeros), so the mixed
    CholGS is the FP64 one."""
    rng = np.random.default_rng(904)
    bv, nb = 8, 4
    X = np.zeros((4 * 300, bv * nb))
    for b in range(nb):
        X[300 * b:300 * (b + 1), bv * b:bv * (b + 1)] = rng.standard_normal((300, bv))
    np.testing.assert_allclose(chfsi.cholgs_mixed(X, bv), chfsi.cholgs(X), rtol=0, atol=1e-14)


def test_cholgs_mixed_error_is_fp32_level():
    rng = np.random.default_rng(905)
    X = rng.standard_normal((3000, 64)) @ np.diag(np.logspace(0, 1, 64))
    Xm = chfsi.cholgs_mixed(X, 16)
    Xd = chfsi.cholgs(X)
    err = np.max(np.abs(Xm - Xd))
    assert 1e-9 < err < 1e-5, err
    orth = np.max(np.abs(Xm.T @ Xm - np.eye(64)))
    assert 1e-10 < orth < 1e-5, orth


def _box_eigvecs():
    L, n_el, p = 9.0, 3, 4
    A = fem.operator_1d(L, n_el, p)
    a, U = np.linalg.eigh(A)
    picks = [(i, j, k) for i in range(4) for j in range(4) for k in range(4)]
    lam = np.array([a[i] + a[j] + a[k] for (i, j, k) in picks])
    order = np.argsort(lam, kind="stable")[:30]
    X = np.stack([np.kron(U[:, picks[t][2]], np.kron(U[:, picks[t][1]], U[:, picks[t][0]])) for t in order], axis=1)
    return A, X, lam[order]


def test_split_rr_mixed_keeps_fp64_accuracy_on_exact_eigenvectors():
    """eq. partialDiagLim1/Lim2: on eigenvectors Hhat is diagonal, the FP32
    coupling blocks are rounding noise, and the fractionally occupied Ritz
    values shift only at second order -- they stay at FP64 accuracy."""
    A, X, lam = _box_eigvecs()
    V = np.zeros(X.shape[0])
    apply = lambda Y: fem.apply_kron(A, V, Y)
    N = X.shape[1]
    # fr0 at a cluster boundary of the box spectrum
    fr0 = max(k for k in range(1, N) if lam[k] - lam[k - 1] > 0.1)
    n_fr = N - fr0
    _, Dm, _ = density.rayleigh_ritz_split(apply, X, n_fr, mixed=True, fr0=fr0)
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(Dm - lam[fr0:])) < 1e-12 * scale
    # the occupied block itself is FP32: its Ritz values are not FP64-accurate
    G = density.projected_split(X, apply(X), fr0)
    Hh = np.tril(G) + np.tril(G, -1).T
    d_oc = np.linalg.eigvalsh(Hh[:fr0, :fr0])
    assert np.max(np.abs(d_oc - lam[:fr0])) > 1e-10 * scale


def test_split_rr_mixed_error_on_random_block_is_fp32_level():
    A, _, _ = _box_eigvecs()
    rng = np.random.default_rng(906)
    n = A.shape[0] ** 3
    V = -2.0 * np.exp(-np.linspace(-3, 3, n) ** 2)
    apply = lambda Y: fem.apply_kron(A, V, Y)
    X = chfsi.cholgs(rng.standard_normal((n, 40)))
    _, D64, _ = density.rayleigh_ritz_split(apply, X, 8, mixed=False)
    _, Dm, _ = density.rayleigh_ritz_split(apply, X, 8, mixed=True)
    scale = np.max(np.abs(D64))
    err = np.max(np.abs(Dm - D64))
    assert 1e-11 * scale < err < 1e-5 * scale, err / scale


@pytest.mark.parametrize("fr0", [0, 17, 40])
def test_projected_split_fp64_block_fp32_elsewhere(fr0):
    rng = np.random.default_rng(907 + fr0)
    X = rng.standard_normal((1200, 40))
    HX = rng.standard_normal((1200, 40)) * 3.0
    G = density.projected_split(X, HX, fr0)
    idx = np.arange(40)
    mask = (idx[:, None] >= fr0) & (idx[None, :] >= fr0)
    worst_r, worst_64 = _check_split_product(X, HX, G, mask)
    if fr0 > 0:
        assert worst_r > 100.0 and worst_64 > 100.0, (worst_r, worst_64)
