"""GPU parity of the matrix-core (MFMA) block products and of whole solves
that run on them, against host float64 references built from the oracle's
quantisation routines (through the C ABI).

The products are sized above the matrix-core thresholds (A X >= 1e8 flops,
A^T X >= 1e9 flops) with ragged row counts and a k that is not a multiple of
the 32-column output tiles.  On the matrix-core path X is packed in A's
type: BF16 by round to nearest even, FP8 e4m3 with one scale amax / 448 per
128 rows of X; the references apply the same packing to X, so a product that
kept X in FP32 (the vector path) would miss the BF16 bound by the rounding
of X (~2^-9)."""
import numpy as np
import pytest

import workloads
from oracle import bki, philox, quant

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_1504_05477_amd as bk


def _cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _rows_fp8(X):
    """Dequantised FP8 copy of X with one scale per 128 rows (all columns)."""
    X = np.asarray(X, dtype=np.float32)
    out = np.empty(X.shape, dtype=np.float64)
    for r0 in range(0, X.shape[0], 128):
        blk = X[r0:r0 + 128]
        am = np.float32(np.max(np.abs(blk))) if blk.size else np.float32(0)
        s = np.float32(am / np.float32(448.0)) if am > 0 else np.float32(1.0)
        out[r0:r0 + 128] = quant.e4m3_decode(quant.e4m3_encode(blk / s)) * np.float64(s)
    return out


def _operands(prec, A, X):
    """(device A in its storage type, its scales, dequantised A, packed X)."""
    Ag = _cuda(A)
    if prec == "f32":
        return Ag, None, A.astype(np.float64), X.astype(np.float64)
    if prec == "bf16":
        Aq = bk.quantize(Ag, "bf16")
        bits = Aq.cpu().view(torch.int16).numpy().view(np.uint16)
        Ad = quant.bf16_decode(bits).astype(np.float64)
        Xd = quant.bf16_decode(quant.bf16_round(X)).astype(np.float64)
        return Aq, None, Ad, Xd
    codes, sc = bk.quantize(Ag, "fp8")
    Ad = quant.dequantize_fp8_tiles(codes.cpu().numpy().view(np.uint8), sc.cpu().numpy())
    return codes, sc, Ad, _rows_fp8(X)


# k = 200: A X on 256-column workgroups (N > 128), the second column half
# ragged (72 of its 128 columns valid)
@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("k", [52, 200])
def test_mfma_block_products(prec, trans, k):
    rng = np.random.default_rng(17)
    # A^T X: 16 column tiles x 32 row splits = 512 workgroups, the smallest
    # FP32 grid that stays on the matrix cores
    n, d = (20000, 2048) if trans else (1500, 1024)
    A = rng.standard_normal((n, d)).astype(np.float32)
    X = rng.standard_normal((n if trans else d, k)).astype(np.float32)
    Aq, sc, Ad, Xd = _operands(prec, A, X)
    Y = bk.dense_product(Aq, _cuda(X), trans=trans, a_scales=sc).cpu().numpy()
    ref = (Ad.T @ Xd) if trans else (Ad @ Xd)
    bound = (np.abs(Ad).T @ np.abs(Xd)) if trans else (np.abs(Ad) @ np.abs(Xd))
    err = np.abs(Y - ref) / bound
    print(f"{prec} trans={trans} n={n} d={d} k={k}: max |err| / (|A||X|) = {err.max():.2e}")
    assert err.max() < 1e-5 if trans else err.max() < 2e-5


@pytest.mark.parametrize("prec", ["plain", "plain_fp32_cores", "bf16", "fp8"])
def test_svd_dense_on_matrix_cores(prec):
    # both block products above the thresholds (2 n d k >= 1e9)
    n, d, k, q = 8192, 2048, 32, 4
    sv = workloads.spectrum("inv", d)
    A = workloads.planted_dense(n, d, sv, 23).astype(np.float32)
    ref = bki.block_krylov(A.astype(np.float64),
                           philox.gaussian(33, d, k).astype(np.float32).astype(np.float64),
                           k, q, tau=1e-5)
    Ag = _cuda(A)
    if prec.startswith("plain"):
        # FP32 products as BF16 limbs (default) or on the FP32 matrix cores
        res = bk.svd_dense(Ag, k, q, seed=33,
                           fp32_products="cores" if prec.endswith("cores") else "limbs")
        tol = 1e-5
    elif prec == "bf16":
        res = bk.svd_dense(bk.quantize(Ag, "bf16"), k, q, seed=33, A_master=Ag)
        tol = 1e-3
    else:
        codes, sc = bk.quantize(Ag, "fp8")
        res = bk.svd_dense(codes, k, q, seed=33, a_scales=sc, A_master=Ag)
        tol = 1e-3
    rel = np.abs(res.sigma.cpu().numpy() - ref.sigma) / ref.sigma
    Z = res.Z.cpu().numpy()
    orth = np.abs(Z.T @ Z - np.eye(k)).max()
    print(f"{prec}: max Ritz rel err {rel.max():.2e}, |Z^T Z - I| {orth:.1e}")
    assert rel.max() <= tol, rel.max()
    assert orth < 1e-4


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_transposed_copy_is_the_transpose(prec):
    # ragged in both dimensions: partial 128 x 128 tiles on both edges
    rng = np.random.default_rng(19)
    A = (rng.standard_normal((1000, 700)) * np.exp(rng.uniform(-3, 3, (1000, 1)))).astype(
        np.float32)
    Ag = _cuda(A)
    if prec == "bf16":
        Aq, At = bk.quantize(Ag, "bf16"), bk.quantize(Ag, "bf16", transposed=True)
        assert tuple(At.shape) == (700, 1000)
        assert torch.equal(At.view(torch.int16), Aq.t().contiguous().view(torch.int16))
    else:
        (Aq, sc), (At, sct) = bk.quantize(Ag, "fp8"), bk.quantize(Ag, "fp8", transposed=True)
        assert tuple(At.shape) == (700, 1000) and tuple(sct.shape) == (6, 8)
        assert torch.equal(At, Aq.t().contiguous())
        assert torch.equal(sct, sc.t().contiguous())
        # and A^T X read row by row from the copy equals the dequantised A^T X
        X = rng.standard_normal((1000, 40)).astype(np.float32)
        Y = bk.dense_product(At, _cuda(X), a_scales=sct).cpu().numpy()
        Ad = quant.dequantize_fp8_tiles(Aq.cpu().numpy().view(np.uint8), sc.cpu().numpy())
        ref = Ad.T @ X.astype(np.float64)
        err = np.abs(Y - ref) / (np.abs(Ad).T @ np.abs(X.astype(np.float64)))
        assert err.max() < 1e-5, err.max()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("n", [8192, 8000])
def test_svd_dense_with_transposed_copy(prec, n):
    # A^T Y on the transposed copy: the A X-form matrix-core kernel (n a
    # multiple of its 128-value chunks) or the vector kernel (n = 8000)
    d, k, q = 2048, 32, 4
    A = workloads.planted_dense(n, d, workloads.spectrum("inv", d), 23).astype(np.float32)
    ref = bki.block_krylov(A.astype(np.float64),
                           philox.gaussian(33, d, k).astype(np.float32).astype(np.float64),
                           k, q, tau=1e-5)
    Ag = _cuda(A)
    if prec == "bf16":
        Aq, At = bk.quantize(Ag, "bf16"), bk.quantize(Ag, "bf16", transposed=True)
        res = bk.svd_dense(Aq, k, q, seed=33, A_master=Ag, A_t=At)
        res0 = bk.svd_dense(Aq, k, q, seed=33, A_master=Ag)
    else:
        (Aq, sc), (At, sct) = bk.quantize(Ag, "fp8"), bk.quantize(Ag, "fp8", transposed=True)
        res = bk.svd_dense(Aq, k, q, seed=33, a_scales=sc, A_master=Ag, A_t=At, at_scales=sct)
        res0 = bk.svd_dense(Aq, k, q, seed=33, a_scales=sc, A_master=Ag)
    s, s0 = res.sigma.cpu().numpy(), res0.sigma.cpu().numpy()
    rel = np.abs(s - ref.sigma) / ref.sigma
    print(f"{prec} n={n}: Ritz rel err {rel.max():.2e} (without the copy "
          f"{(np.abs(s0 - ref.sigma) / ref.sigma).max():.2e}), q_eff {res.info['q_eff']}")
    assert rel.max() <= 1e-3
    assert res.info["q_eff"] == res0.info["q_eff"]
    Z = res.Z.cpu().numpy()
    assert np.abs(Z.T @ Z - np.eye(k)).max() < 1e-4
