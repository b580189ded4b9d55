"""Every tile variant of the n x n by n x r product kernels against numpy.

FP64: 1e-13 relative (Frobenius).  FP32 and BF16 operands are rounded on the
host exactly as the library stores them (round to nearest even), the skinny
operand as the kernels carry it (FP32: one rounding; BF16: a hi + lo pair of
bf16), and the reference product is then taken in FP64: what remains is FP32
accumulation, bounded here by 1e-5 relative.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import bf16_tiles, product  # noqa: E402

TILES = {"fp64": [(1, 4), (1, 8), (2, 4), (2, 8), (4, 2), (4, 4)],
         "fp32": [(1, 4), (1, 8), (2, 4), (2, 8), (4, 4)],
         "bf16": [(1, 4), (2, 2), (2, 4), (4, 2)]}


def _rnd(a, dt):
    return torch.from_numpy(a).to(dt).to(torch.float64).numpy()


def _split_bf16(a):
    hi = _rnd(_rnd(a, torch.float32), torch.bfloat16)
    return hi + _rnd(_rnd(a - hi, torch.float32), torch.bfloat16)


def _case(n, r, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, n))
    X = rng.standard_normal((n, r))
    scale = rng.uniform(0.5, 2.0, n)
    return U, X, scale


@pytest.mark.parametrize("elt", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,r", [(37, 5), (300, 17), (1000, 40), (777, 64), (129, 33)])
def test_product_all_tiles(elt, n, r):
    U, X, scale = _case(n, r, n + r)
    Xd = torch.from_numpy(X).cuda()
    sd = torch.from_numpy(scale).cuda()
    if elt == "fp64":
        Ud = torch.from_numpy(U).cuda()
        Ur, opx, gate, transes = U, (lambda a: a), 1e-13, (False, True)
    elif elt == "fp32":
        Ud = torch.from_numpy(U).cuda().float()
        Ur, opx, gate, transes = _rnd(U, torch.float32), (lambda a: _rnd(a, torch.float32)), \
            1e-5, (False, True)
    else:
        ld = (n + 255) // 256 * 256
        Ud = torch.zeros(n, ld, dtype=torch.bfloat16, device="cuda")
        Ud[:, :n] = torch.from_numpy(U).cuda().to(torch.bfloat16)
        Ur, opx, gate, transes = _rnd(U, torch.bfloat16), _split_bf16, 1e-5, (False,)
    Ut = bf16_tiles(Ud) if elt == "bf16" else None
    for trans in transes:
        A = Ur.T if trans else Ur
        want = A @ opx(scale[:, None] * X)
        for tile in TILES[elt]:
            for ks in (0, 1, 3):
                got = product(Ud, Xd, elt, trans, tile, ks, sd)
                gh = got.cpu().numpy()
                err = np.linalg.norm(gh - want) / np.linalg.norm(want)
                assert err <= gate, (elt, trans, tile, ks, err)
                # every row on its own (rows of a random U have similar norms):
                # a wrong tail row or padding column cannot hide in the norm
                rerr = np.max(np.linalg.norm(gh - want, axis=1) / np.linalg.norm(want, axis=1))
                assert rerr <= 10 * gate, (elt, trans, tile, ks, rerr)
                if Ut is not None:
                    # the tiled layout changes addresses only: identical results
                    got_t = product(Ut, Xd, "bf16_tiled", False, tile, ks, sd)
                    assert torch.equal(got_t, got), (tile, ks)


def test_product_rejects_bad_tiles_and_shapes():
    X = torch.zeros(40, 8, dtype=torch.float64, device="cuda")
    U = torch.zeros(40, 40, dtype=torch.float64, device="cuda")
    with pytest.raises(C.CphifiError):
        product(U, X, "fp64", False, (3, 4))
    Ub = torch.zeros(40, 40, dtype=torch.bfloat16, device="cuda")  # stride < 128
    with pytest.raises(C.CphifiError):
        product(Ub, X, "bf16", False, (2, 4))
    Ub = torch.zeros(40, 136, dtype=torch.bfloat16, device="cuda")  # tiled: stride % 64 != 0
    with pytest.raises(C.CphifiError):
        product(Ub, X, "bf16_tiled", False, (2, 4))


@pytest.mark.parametrize("n,r", [(10300, 40), (12345, 5)])
def test_fp64_stream_k_product(n, r, monkeypatch):
    """The stream-K form of the transposed FP64 product (CPHIFI_F64_STREAMK=1;
    used when the split-K grid leaves resident slots idle, which these sizes
    do): every row against numpy, for each 4x4x4 tile shape."""
    monkeypatch.setenv("CPHIFI_F64_STREAMK", "1")
    U, X, scale = _case(n, r, n + r)
    want = U.T @ (scale[:, None] * X)
    Ud = torch.from_numpy(U).cuda()
    Xd = torch.from_numpy(X).cuda()
    sd = torch.from_numpy(scale).cuda()
    for tile in [(4, 2), (2, 4), (1, 8)]:
        gh = product(Ud, Xd, "fp64", True, tile, 0, sd).cpu().numpy()
        rerr = np.max(np.linalg.norm(gh - want, axis=1) / np.linalg.norm(want, axis=1))
        assert rerr <= 1e-12, (tile, rerr)


@pytest.mark.parametrize("n,r", [(5000, 40), (12345, 7)])
def test_bf16_stream_k_product(n, r, monkeypatch):
    """The stream-K form of the tiled BF16 product (CPHIFI_BF16_STREAMK=1;
    these sizes leave CUs idle under split-K, so the plan takes it, with up to
    14 contributors per row block): every row against numpy on the rounded
    operands."""
    monkeypatch.setenv("CPHIFI_BF16_STREAMK", "1")
    U, X, scale = _case(n, r, n + r)
    ld = (n + 255) // 256 * 256
    Ud = torch.zeros(n, ld, dtype=torch.bfloat16, device="cuda")
    Ud[:, :n] = torch.from_numpy(U).cuda().to(torch.bfloat16)
    want = _rnd(U, torch.bfloat16) @ _split_bf16(scale[:, None] * X)
    del U
    Xd = torch.from_numpy(X).cuda()
    sd = torch.from_numpy(scale).cuda()
    gh = product(bf16_tiles(Ud), Xd, "bf16_tiled", False, (4, 2), 0, sd).cpu().numpy()
    assert np.linalg.norm(gh - want) / np.linalg.norm(want) <= 1e-5
    rerr = np.max(np.linalg.norm(gh - want, axis=1) / np.linalg.norm(want, axis=1))
    assert rerr <= 1e-4, rerr


@pytest.mark.parametrize("count,blocks", [(1 << 20, 64), (3 * (1 << 20) + 6, 1000)])
def test_stream_read_reads_every_element(count, blocks):
    """The streaming-read helper (the achievable-bandwidth probe) visits every
    element once: the partial sums add up to the buffer's sum (integer values,
    so every order of addition gives the exact total)."""
    g = torch.Generator(device="cuda").manual_seed(9)
    buf = torch.randint(-1000, 1000, (count,), generator=g, device="cuda").to(torch.float64)
    part = torch.zeros(blocks, dtype=torch.float64, device="cuda")
    C.cphifi_stream_read(buf.data_ptr(), count * 8, blocks, part.data_ptr(), 0)
    torch.cuda.synchronize()
    assert float(part.sum()) == float(buf.sum())
    with pytest.raises(C.CphifiError):
        C.cphifi_stream_read(buf.data_ptr(), count * 8 - 8, blocks, part.data_ptr(), 0)
