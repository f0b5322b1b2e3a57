"""diaq_expect_noalloc, the allocation-free expectation value: through the C
ABI, against diaq_expect on the same inputs (same kernels and summation
order, so bit for bit) and against the oracle, on consecutive calls whose
second input is smaller than the first (the shared static partial-sum array
keeps the first call's contents), in complex128 and complex64, with a
matrix of more diagonals than the kernel arguments hold (device table), an
empty matrix, and a product beyond the static array's size."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _hea_terms(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n - 1)
    b = rng.standard_normal(n)
    return [(0, (1 << i) | (1 << (i + 1)), float(a[i])) for i in range(n - 1)] + \
           [(1 << i, 0, float(b[i])) for i in range(n)]


def _noalloc(H, psi, phi=None):
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda:0")
    D.expect_noalloc(H, psi, out, phi)
    torch.cuda.synchronize()
    v = out.cpu().numpy()
    return complex(v[0], v[1])


def test_noalloc_matches_expect_on_consecutive_calls():
    # first call: n = 20, 41 diagonals (device descriptor table), <psi|H|psi>
    n1 = 20
    terms1 = _hea_terms(n1, 1)
    H1 = D.from_pauli_sum(n1, terms1)
    x1 = W.random_state(n1, 11)
    psi1 = to_dev(x1)
    got1 = _noalloc(H1, psi1)
    want1 = D.expect(H1, psi1)
    assert got1 == want1
    ref1 = orc.expect(n1, terms1, x1)
    assert abs(got1 - ref1) <= 1e-12
    # second call, smaller: n = 12, 3 diagonals, <psi|H|phi> with phi != psi
    n2 = 12
    terms2 = [(1 << 3, 1 << 5, 0.7), (0, 0b1010, -1.3), (1 << 11, 0, 0.4)]
    H2 = D.from_pauli_sum(n2, terms2)
    x2, y2 = W.random_state(n2, 12), W.random_state(n2, 13)
    psi2, phi2 = to_dev(x2), to_dev(y2)
    got2 = _noalloc(H2, psi2, phi2)
    assert got2 == D.expect(H2, psi2, phi2)
    assert abs(got2 - orc.expect(n2, terms2, x2, y2)) <= 1e-12
    # and the first input again: nothing of the smaller call carries over
    assert _noalloc(H1, psi1) == want1


def test_noalloc_complex64_and_caller_matrix():
    rng = np.random.default_rng(5)
    n = 14
    N = 1 << n
    diags = {d: rng.standard_normal(N - abs(d)) + 1j * rng.standard_normal(N - abs(d)) for d in (-700, -1, 0, 3, 4096)}
    x = W.random_state(n, 14)
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-4)):
        A = D.from_dense_diagonals(n, diags, dtype=dtype)
        psi = to_dev(x, dtype)
        got = _noalloc(A, psi)
        assert got == D.expect(A, psi)
        o, s, v = orc.pack_dia(sorted(diags), [diags[d] for d in sorted(diags)])
        ref = orc.inner(x.astype(dtype_np(dtype)).astype(np.complex128),
                        orc.dia_spmv(N, o, s, v, x.astype(dtype_np(dtype)).astype(np.complex128)))
        assert abs(got - ref) <= tol * max(1.0, abs(ref))


def dtype_np(dtype):
    return np.complex128 if dtype == torch.complex128 else np.complex64


def test_noalloc_empty_matrix_and_size_limit():
    n = 10
    A = D.from_dense_diagonals(n, {})
    psi = to_dev(W.random_state(n, 1))
    assert _noalloc(A, psi) == 0
    # 2^29 rows need 2^21 partial sums at one row per lane: rejected before
    # any launch, the output untouched
    ctx = D.context()
    saved = D.get_tuning(ctx)
    D.set_tuning(ctx, spmv_rows=1)
    try:
        _size_limit()
    finally:
        D.set_tuning(ctx, **saved)


def _size_limit():
    n = 29
    Z = D.from_pauli_sum(n, [(0, 1, 1.0)])
    big = torch.zeros(1 << n, dtype=torch.complex128, device="cuda:0")
    out = torch.full((2,), 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(D.DiaqError) as ei:
        D.expect_noalloc(Z, big, out)
    assert ei.value.status == 5  # DIAQ_ERR_UNSUPPORTED
    assert out.cpu().tolist() == [7.0, 7.0]
    del big, Z


def test_noalloc_allocates_nothing():
    n = 18
    terms = _hea_terms(n, 3)
    H = D.from_pauli_sum(n, terms)
    psi = to_dev(W.random_state(n, 18))
    out = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    D.expect_noalloc(H, psi, out)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        D.expect_noalloc(H, psi, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert complex(*out.cpu().tolist()) == D.expect(H, psi)
