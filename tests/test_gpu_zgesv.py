"""The batched linear solve of Sec. II (ZGESV with N right-hand sides) through
wpccc_zgesv_batched, against LAPACK's ZGESV (numpy.linalg.solve).

Bar: max|X_gpu - X_lapack| <= 200 n eps cond(A) max|X|: both are backward
stable LU solves with partial pivoting (the same pivot rule, so the same
factors up to the order of the sums), whose forward errors are bounded by
cond(A) times a small multiple of n eps.
"""
import numpy as np
import pytest
import torch

import paper_2403_04252_amd as W

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


def cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def solve_gpu(A, B):
    """A, B: numpy [batch, n, n] (A row-major as in numpy)."""
    At = torch.as_tensor(np.ascontiguousarray(A.transpose(0, 2, 1)), device="cuda")
    Bt = torch.as_tensor(np.ascontiguousarray(B), device="cuda")
    X = torch.empty_like(Bt)
    W.wpccc_zgesv_batched(At, Bt, X)
    torch.cuda.synchronize()
    return X.cpu().numpy()


@pytest.mark.parametrize("n", [1, 37, 100, 300, 1100])
def test_zgesv_random(n):
    """Random complex systems (ragged against the 32-row blocks and the LU
    panels; n = 1100 takes the 8-column panels of the largest systems), one
    with a zero diagonal so that every column pivots."""
    rng = np.random.default_rng(100 + n)
    batch = 1 if n > 1000 else 3
    A = cplx(rng, batch, n, n)
    if batch > 1 and n > 1:
        A[1][np.arange(n), np.arange(n)] = 0.0
    B = cplx(rng, batch, n, n)
    print(f"zgesv n={n} batch={batch}", flush=True)
    X = solve_gpu(A, B)
    for b in range(batch):
        Xo = np.linalg.solve(A[b], B[b])
        err = np.abs(X[b] - Xo).max()
        bar = 200 * n * EPS * np.linalg.cond(A[b]) * np.abs(Xo).max()
        res = np.abs(A[b] @ X[b] - B[b]).max() / (np.abs(A[b]).max() * np.abs(X[b]).max() * n)
        print(f"  matrix {b}: max|dX| {err:.2e} (bar {bar:.1e}), scaled residual {res:.1e}", flush=True)
        assert err <= bar and res <= 10 * EPS


def test_zgesv_singular_flagged():
    """An exactly zero column in the second matrix of the batch: the LU meets a
    zero pivot there, which the call reports as WPCCC_ESINGULAR naming the
    matrix and column; the other matrices are still solved."""
    rng = np.random.default_rng(7)
    n = 50
    A = cplx(rng, 3, n, n)
    A[1][:, 17] = 0.0
    B = cplx(rng, 3, n, n)
    At = torch.as_tensor(np.ascontiguousarray(A.transpose(0, 2, 1)), device="cuda")
    Bt = torch.as_tensor(B, device="cuda")
    X = torch.empty_like(Bt)
    with pytest.raises(W.WpcccError) as e:
        W.wpccc_zgesv_batched(At, Bt, X)
    torch.cuda.synchronize()
    assert e.value.code == -4
    assert "matrix 1" in str(e.value) and "column 17" in str(e.value), str(e.value)
    Xh = X.cpu().numpy()
    for b in (0, 2):
        assert np.abs(Xh[b] - np.linalg.solve(A[b], B[b])).max() <= 1e-9
    # the library stays usable after the flag
    X2 = solve_gpu(A[[0]], B[[0]])
    assert np.abs(X2[0] - np.linalg.solve(A[0], B[0])).max() <= 1e-9


def test_zgesv_argument_errors():
    A = torch.zeros((1, 4, 4), dtype=torch.complex128, device="cuda")
    lib = W.load_library()
    assert lib.wpccc_zgesv_batched(0, 1, A.data_ptr(), A.data_ptr(), A.data_ptr(), None) == -1
    assert lib.wpccc_zgesv_batched(4, 1, None, A.data_ptr(), A.data_ptr(), None) == -1
    assert lib.wpccc_zgesv_batched(4097, 1, A.data_ptr(), A.data_ptr(), A.data_ptr(), None) == -1
