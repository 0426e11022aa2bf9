"""The warm-start network on the GPU (include/rpmfno.h): the matrix-core GEMM
(bfloat16 operands, FP32 accumulation) exactly on bfloat16-representable
integers and to FP32 accumulation error on rounded operands, and the forward
pass and gradients of the whole network against the FP64 CPU reference
(oracle/fno_ref.py) to bfloat16 accuracy."""
import numpy as np
import pytest

from oracle import fno_ref as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


def t32(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,batch,ta,tb", [(16, 16, 16, 1, 0, 0), (37, 29, 23, 3, 0, 1), (64, 5, 70, 2, 1, 0),
                                               (1, 33, 9, 4, 1, 1), (130, 66, 48, 1, 0, 0)])
def test_gemm_exact_on_small_integers(B, M, N, K, batch, ta, tb):
    """Integer operands in [-8, 8] are exact in bfloat16 and the FP32 sums are
    exact: the matrix-core product must equal numpy's bit for bit (this pins the
    lane layout of the MFMA operands and results), with transposed operands and
    batches given by strides."""
    r = np.random.default_rng(M * 1000 + N)
    A = r.integers(-8, 9, size=(batch, M, K)).astype(np.float64)
    Bm = r.integers(-8, 9, size=(batch, K, N)).astype(np.float64)
    C0 = r.integers(-8, 9, size=(batch, M, N)).astype(np.float64)
    As = np.ascontiguousarray(np.transpose(A, (0, 2, 1))) if ta else A
    Bs = np.ascontiguousarray(np.transpose(Bm, (0, 2, 1))) if tb else Bm
    sA = (M * K, 1, M) if ta else (M * K, K, 1)
    sB = (K * N, 1, K) if tb else (K * N, N, 1)
    dA, dB, dC = t32(As), t32(Bs), t32(C0)
    B.gemm_bf16(dA, sA, dB, sB, dC, (M * N, N, 1), M, N, K, batch, alpha=2.0, beta=-1.0)
    ref = 2.0 * np.einsum("bik,bkj->bij", A, Bm) - C0
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), ref)


def test_gemm_rounded_operands(B):
    r = np.random.default_rng(7)
    M, N, K = 50, 40, 96
    A = r.normal(size=(M, K))
    Bm = r.normal(size=(K, N))
    dC = t32(np.zeros((M, N)))
    B.gemm_bf16(t32(A), (0, K, 1), t32(Bm), (0, N, 1), dC, (0, N, 1), M, N, K)
    ref = bf16_round(A) @ bf16_round(Bm)
    err = np.abs(dC.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err


@pytest.mark.parametrize("shape", [(4, 6, 8), (8, 8, 8)])
def test_network_forward_and_gradients_match_fp64_reference(B, shape):
    import torch

    cfg_t = (2, 36, 8, 2, 4)
    cfg = B.fno_config(*cfg_t)
    params = B.fno_init(cfg, 11)
    # non-zero biases so every term of the gradient is exercised
    p = params.cpu().numpy().astype(np.float64)
    r = np.random.default_rng(5)
    d = F.unpack(p, cfg_t)
    for k in d:
        if k.endswith("_b") or k.startswith("b"):
            d[k][...] = 0.1 * r.normal(size=d[k].shape)
    p = F.pack(d, cfg_t)
    params = t32(p)
    p = params.cpu().numpy().astype(np.float64)  # the float32 values both sides use
    x = r.normal(size=(2, 2) + shape).astype(np.float32)
    dy = r.normal(size=(2, 36) + shape).astype(np.float32)
    y_ref, cache = F.forward(p, cfg_t, x.astype(np.float64))
    g_ref, dx_ref = F.backward(p, cfg_t, cache, dy.astype(np.float64))
    y, ws = B.fno_forward(cfg, params, t32(x))
    g, dx = B.fno_backward(cfg, params, t32(x), t32(dy), ws, want_dx=True)
    torch.cuda.synchronize()
    ey = np.linalg.norm(y.cpu().numpy() - y_ref) / np.linalg.norm(y_ref)
    eg = np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    ex = np.linalg.norm(dx.cpu().numpy() - dx_ref) / np.linalg.norm(dx_ref)
    print(f"forward {ey:.2e} grad {eg:.2e} dx {ex:.2e}", flush=True)
    # bfloat16 operands: about 2^-9 relative per product, a few products deep
    assert ey < 1e-2 and eg < 3e-2 and ex < 3e-2, (ey, eg, ex)
    # every parameter block individually
    gg = F.unpack(g.cpu().numpy().astype(np.float64), cfg_t)
    gr = F.unpack(g_ref, cfg_t)
    for k in gr:
        nrm = np.linalg.norm(gr[k])
        if nrm > 0:
            assert np.linalg.norm(gg[k] - gr[k]) / nrm < 5e-2, k
