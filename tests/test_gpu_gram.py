"""GPU parity of the tall-skinny Gram product behind the true-residual evaluation (sylv_gram):
C = A^T B for K x M and K x N row-major FP64 operands, against NumPy FP64 products of the same
seeded inputs.

* The shapes the 1024^2 Lyapunov residual forms for every 16384-row chunk at rank 2893 (the
  symmetric basis Gram and the 2893 x 2894 cross Gram): 128 x 128 tiles, whole tiles in rounds
  of 512 workgroups plus the remainder split over K (stream-K) and summed by the fix-up kernel.
  Checked on sampled output rows (every column tile, the rows at tile borders and the last rows)
  against exact FP64 products of those rows, for symmetry (the mirror), and for bit-identical
  repeats (the order of every sum is fixed).
* A ragged case (K not a multiple of the slab depth, the leading dimension not a multiple of
  128, so the last column tile reads past M), accumulation (C += A^T B), too little scratch
  (the product falls back to 64 x 64 tiles) and none, and small shapes on the 64 x 64 paths.

Tolerance: |C - C_ref| <= 1e-13 K max|A| max|B| per entry, far above the FP64 rounding of
either summation order (about sqrt(K) eps |a| |b|) and far below any indexing mistake (an
entry of the wrong tile or row is off by O(sqrt(K)))."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def _operand(rng, K, cols, ld):
    a = np.zeros((K, ld))
    a[:, :cols] = rng.standard_normal((K, cols))
    # columns past the operand hold large finite values: they must not reach any stored entry
    a[:, cols:] = 1e6
    return a


def _sample_rows(M, rng, n=24):
    rows = {0, 1, M - 1, M - 2}
    for b in range(128, M, 128):
        rows.update((b - 1, b))
    rows = sorted(r for r in rows if 0 <= r < M)
    extra = rng.choice(M, size=min(n, M), replace=False)
    return np.unique(np.concatenate([rows, extra]))


def _check(got, A, B, M, N, K, rows, C0=None):
    ref = A[:, rows].T @ B[:, :N]
    if C0 is not None:
        ref = ref + C0[rows, :N]
    tol = 1e-13 * K * np.abs(A[:, :M]).max() * np.abs(B[:, :N]).max()
    err = np.abs(got[rows, :N] - ref).max()
    assert err <= tol, (err, tol)


def _run(sylv, M, N, K, lda, ldb, symmetric, seed, work="full", accumulate=False):
    rng = np.random.default_rng(seed)
    A = _operand(rng, K, M, lda)
    B = A if symmetric else _operand(rng, K, N, ldb)
    ldc = N + 5
    C0 = rng.standard_normal((M, ldc)) if accumulate else None
    dA = torch.as_tensor(A, device="cuda")
    dB = dA if symmetric else torch.as_tensor(B, device="cuda")
    dC = torch.as_tensor(C0, device="cuda") if accumulate else \
        torch.full((M, ldc), np.nan, dtype=torch.float64, device="cuda")
    need = sylv.sylv_gram_work_bytes(M, N, K)
    nbytes = {"full": need, "small": 2 * 64 * 64 * 8 * 3, "none": 0}[work]
    dW = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device="cuda") if nbytes else None
    print(f"sylv_gram M={M} N={N} K={K} lda={lda} symmetric={symmetric} work={work}", flush=True)
    sylv.sylv_gram(M, N, K, dA, lda, dB, ldb, dC, ldc, symmetric=symmetric,
                   accumulate=accumulate, work=dW, work_bytes=nbytes)
    got = dC.cpu().numpy()
    return A, B, C0, got, (dA, dB, dC, dW, nbytes, ldc)


@pytest.mark.parametrize("M,N,symmetric", [(2893, 2893, True), (2893, 2894, False)])
def test_residual_chunk_grams(sylv, M, N, symmetric):
    K, ld = 16384, 4032
    A, B, _, got, (dA, dB, dC, dW, nbytes, ldc) = _run(sylv, M, N, K, ld, ld, symmetric, M + N)
    rng = np.random.default_rng(5)
    rows = _sample_rows(M, rng)
    _check(got, A, B, M, N, K, rows)
    assert np.isfinite(got[:, :N]).all()
    assert np.isnan(got[:, N:]).all()  # nothing written past N
    if symmetric:
        assert np.array_equal(got[:, :N], got[:, :N].T)
    # a repeat gives the same bits
    sylv.sylv_gram(M, N, K, dA, ld, dB, ld, dC, ldc, symmetric=symmetric, work=dW,
                   work_bytes=nbytes)
    assert np.array_equal(dC.cpu().numpy()[:, :N], got[:, :N])


@pytest.mark.parametrize("work", ["full", "small", "none"])
def test_ragged_gram_and_scratch_sizes(sylv, work):
    # 22 x 22 tiles of 128: K % 16 = 11 and lda = 2752 (the last column tile reads past lda)
    M, N, K = 2700, 2750, 16379
    lda, ldb = 2752, 2752 + 64
    A, B, _, got, _ = _run(sylv, M, N, K, lda, ldb, False, 77, work=work)
    _check(got, A, B, M, N, K, _sample_rows(M, np.random.default_rng(6)))
    assert np.isfinite(got[:, :N]).all()


def test_gram_accumulates(sylv):
    M, N, K = 2750, 2750, 4099
    A, B, C0, got, _ = _run(sylv, M, N, K, 2816, 2816, False, 88, accumulate=True)
    _check(got, A, B, M, N, K, _sample_rows(M, np.random.default_rng(7)), C0=C0)


@pytest.mark.parametrize("M,N,K,symmetric", [(1, 1, 1, True), (70, 53, 37, False),
                                             (300, 300, 5000, True), (640, 130, 20000, False),
                                             (1300, 1300, 16384, True)])
def test_small_grams(sylv, M, N, K, symmetric):
    lda = (M + 63) // 64 * 64
    ldb = lda if symmetric else (N + 63) // 64 * 64
    A, B, _, got, _ = _run(sylv, M, N, K, lda, ldb, symmetric, M * 7 + K)
    rows = np.arange(M) if M <= 300 else _sample_rows(M, np.random.default_rng(8))
    _check(got, A, B, M, N, K, rows)


def test_gram_argument_errors(sylv):
    d = torch.zeros(64 * 64, dtype=torch.float64, device="cuda")
    with pytest.raises(sylv.SylvError):
        sylv.sylv_gram(10, 10, 0, d, 64, d, 64, d, 10)  # K = 0
    with pytest.raises(sylv.SylvError):
        sylv.sylv_gram(10, 10, 5, d, 60, d, 64, d, 10)  # lda below 64
    with pytest.raises(sylv.SylvError):
        sylv.sylv_gram(10, 12, 5, d, 64, d, 64, d, 12, symmetric=True)  # M != N
    assert sylv.sylv_gram_work_bytes(0, 5, 5) == 0
    assert sylv.sylv_gram_work_bytes(3000, 3000, 16384) >= 2 * 512 * 128 * 128 * 8
