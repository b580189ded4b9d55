"""cphifi_product_static (no workspace: split-K partials in the library's static
device scratch) against cphifi_product (caller workspace), through the C ABI.

Two calls in a row, the second smaller, must give the existing entry point's
results: bit for bit where both take the same split (same kernels, same
summation order), within the FP64 product bar (1e-13 relative) where the
static entry reduces the split to fit its scratch.  A product whose partials
cannot fit is rejected with INVALID_ARG.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import bf16_tiles, product  # noqa: E402


def _stream():
    return torch.cuda.current_stream().cuda_stream


def static_product(U, X, elt, trans, tile, ksplit=0, xscale=None):
    e = {"fp64": C.ELT_F64, "fp32": C.ELT_F32, "bf16_tiled": C.ELT_BF16_TILED}[elt]
    n, r = X.shape
    Y = torch.full((n, r), float("nan"), dtype=torch.float64, device=X.device)
    C.cphifi_product_static(e, int(trans), tile[0], tile[1], ksplit, n, U.data_ptr(),
                            U.stride(0), X.data_ptr(), r,
                            None if xscale is None else xscale.data_ptr(), Y.data_ptr(),
                            _stream())
    return Y


def _operands(n, r, seed, elt):
    g = torch.Generator(device="cuda").manual_seed(seed)
    U = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    X = torch.randn(n, r, dtype=torch.float64, device="cuda", generator=g)
    s = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) + 0.5
    if elt == "fp32":
        U = U.float()
    elif elt == "bf16_tiled":
        ld = (n + 255) // 256 * 256
        Ub = torch.zeros(n, ld, dtype=torch.bfloat16, device="cuda")
        Ub[:, :n] = U.to(torch.bfloat16)
        U = bf16_tiles(Ub)
    return U, X, s


def test_static_scratch_size_is_stated():
    assert C.cphifi_product_static_max_bytes() == 64 << 20


def test_two_calls_in_a_row_match_the_workspace_entry():
    # first call: FP64 transposed, n = 3000, r = 40 (the split fits: identical)
    U, X, s = _operands(3000, 40, 1, "fp64")
    want = product(U, X, "fp64", True, (4, 2), 0, s)
    got = static_product(U, X, "fp64", True, (4, 2), 0, s)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # second call, smaller, other element type: the scratch keeps the last
    # call's contents, which must not leak into this one
    U2, X2, s2 = _operands(700, 9, 2, "bf16_tiled")
    want2 = product(U2, X2, "bf16_tiled", False, (4, 2), 0, s2)
    got2 = static_product(U2, X2, "bf16_tiled", False, (4, 2), 0, s2)
    torch.cuda.synchronize()
    assert torch.equal(got2, want2)
    U3, X3, _ = _operands(257, 17, 3, "fp32")
    want3 = product(U3, X3, "fp32", False, (2, 4), 3)
    got3 = static_product(U3, X3, "fp32", False, (2, 4), 3)
    torch.cuda.synchronize()
    assert torch.equal(got3, want3)


def test_large_product_reduces_its_split_to_fit():
    n, r = 20000, 64
    U, X, _ = _operands(n, r, 4, "fp64")
    want = product(U, X, "fp64", True, (1, 8), 16)
    got = static_product(U, X, "fp64", True, (1, 8), 0)
    torch.cuda.synchronize()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    assert np.linalg.norm(g - w) <= 1e-13 * np.linalg.norm(w)
    assert np.max(np.linalg.norm(g - w, axis=1) / np.linalg.norm(w, axis=1)) <= 1e-12
    # an explicit split whose partials exceed the scratch is refused
    with pytest.raises(C.CphifiError) as ei:
        static_product(U, X, "fp64", True, (1, 8), 16)
    assert ei.value.status == C.INVALID_ARG
    assert "static scratch" in str(ei.value)
