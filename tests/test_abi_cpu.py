"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad descriptions before touching a GPU."""

import ctypes

import pytest

from paper_2603_25691_amd import cphifi as c


def test_library_exports_every_declared_function():
    names = c.declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(c.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), f"{name} declared in cphifi.h but not exported"


def test_version_and_status_strings():
    assert "gfx950" in c.version()
    assert c.status_string(c.OK) == "CPHIFI_OK"
    assert c.status_string(c.NOT_CONVERGED) == "CPHIFI_NOT_CONVERGED"
    assert c.status_string(999) == "CPHIFI_UNKNOWN"


def test_struct_layout_matches_header():
    # int64 x6 + double x5 + int32 x6 = 112 bytes; 10 pointers; info 48 bytes
    assert ctypes.sizeof(c.cphifi_ui_desc) == 112
    assert ctypes.sizeof(c.cphifi_ui_inputs) == 80
    assert ctypes.sizeof(c.cphifi_solve_info) == 48


def test_workspace_holds_transposed_eigenvectors_from_4096():
    n, r = 5000, 10
    base = c.cphifi_ui_workspace_bytes(c.make_desc(n, r, 100000, 100, 20))
    lean = c.cphifi_ui_workspace_bytes(c.make_desc(n, r, 100000, 100, 20,
                                                   flags=c.FLAG_NO_UKT_COPY))
    assert base - lean >= 8 * n * n
    assert base - lean <= 8 * n * n + 512
    small = c.make_desc(4095, r, 100000, 100, 20)
    assert c.cphifi_ui_workspace_bytes(small) == c.cphifi_ui_workspace_bytes(
        c.make_desc(4095, r, 100000, 100, 20, flags=c.FLAG_NO_UKT_COPY))


def test_bf16_workspace_holds_fp32_eigenvectors_from_4096():
    """MIXED_BF16 plans with n >= 4096 keep U_K^T in FP32 too (row pitch
    round_up(n, 256)) for the early refinement residuals, unless
    CPHIFI_FLAG_FP64_RESIDUALS; other precisions never do."""
    n, r = 5000, 10
    ldl = -(-n // 256) * 256

    def ws(nn, precision, flags=0):
        return c.cphifi_ui_workspace_bytes(c.make_desc(nn, r, 100000, 100, 20,
                                                       precision=precision, flags=flags))
    diff = ws(n, c.MIXED_BF16) - ws(n, c.MIXED_BF16, c.FLAG_FP64_RESIDUALS)
    assert 4 * n * ldl <= diff <= 4 * n * ldl + 512
    for prec in (c.FP64, c.MIXED_FP32):
        assert ws(n, prec) == ws(n, prec, c.FLAG_FP64_RESIDUALS)
    assert ws(4095, c.MIXED_BF16) == ws(4095, c.MIXED_BF16, c.FLAG_FP64_RESIDUALS)


def test_workspace_grows_with_problem_and_precision():
    small = c.cphifi_ui_workspace_bytes(c.make_desc(200, 5, 2000, 20, 10))
    big = c.cphifi_ui_workspace_bytes(c.make_desc(3000, 40, 600000, 100, 200))
    assert 0 < small < big
    fp64 = c.cphifi_ui_workspace_bytes(c.make_desc(3000, 40, 600000, 100, 200))
    bf16 = c.cphifi_ui_workspace_bytes(c.make_desc(3000, 40, 600000, 100, 200,
                                                   precision=c.MIXED_BF16))
    fp32 = c.cphifi_ui_workspace_bytes(c.make_desc(3000, 40, 600000, 100, 200,
                                                   precision=c.MIXED_FP32))
    # the low-precision copies of U_K: 2 bf16 copies, or 1 fp32 copy
    ldl = (3000 + 255) // 256 * 256
    assert bf16 - fp64 >= 2 * 2 * 3000 * ldl
    assert fp32 - fp64 >= 4 * 3000 * ldl


@pytest.mark.parametrize("field,value", [
    ("n", 0), ("r", 0), ("r", 65), ("q", -1), ("lambda_", 0.0), ("rho", -1.0), ("rho", 0.0),
    ("tol", 0.0), ("precision", 7), ("ldk", 5),
])
def test_invalid_descriptions_are_rejected(field, value):
    d = c.make_desc(200, 5, 2000, 20, 10)
    setattr(d, field, value)
    with pytest.raises(c.CphifiError) as ei:
        c.cphifi_ui_workspace_bytes(d)
    assert ei.value.status == c.INVALID_ARG
    assert c.last_error() != ""


def test_no_precond_flag_is_fp64_only():
    d = c.make_desc(200, 5, 2000, 20, 10, precision=c.MIXED_BF16, flags=c.FLAG_NO_PRECOND)
    with pytest.raises(c.CphifiError):
        c.cphifi_ui_workspace_bytes(d)


def test_plan_create_rejects_missing_pointers_without_gpu():
    d = c.make_desc(200, 5, 2000, 20, 10)
    inp = c.make_inputs()  # all NULL
    with pytest.raises(c.CphifiError) as ei:
        c.cphifi_ui_plan_create(d, inp, 0, 0, 0)
    assert ei.value.status == c.INVALID_ARG


def test_oracle_and_library_share_no_code():
    """The product package never imports the oracle, and vice versa."""
    import pathlib

    root = pathlib.Path(c.__file__).resolve().parents[1]
    for f in (root / "paper_2603_25691_amd").rglob("*.py"):
        txt = f.read_text()
        assert "import oracle" not in txt and "from oracle" not in txt, f
    for f in (root / "oracle").rglob("*.py"):
        txt = f.read_text()
        assert "import paper_2603_25691_amd" not in txt, f
        assert "from paper_2603_25691_amd" not in txt, f


def _bf16_desc(n=600, r=10, **kw):
    return c.make_desc(n, r, n * 20, 20, 20, lam=1e-4, tol=1e-8, precision=c.MIXED_BF16, **kw)


def test_batch_workspace_is_members_plus_scalars():
    """The batch adds only its control words, per-member scalars and the grid
    barrier's flags (one 64-byte line for each of up to 2048 workgroups) to
    the members' own workspaces."""
    descs = [_bf16_desc(600, 10), _bf16_desc(1500, 40), _bf16_desc(77, 3)]
    total = c.cphifi_batch_workspace_bytes(descs)
    members = sum(c.cphifi_ui_workspace_bytes(d) for d in descs)
    assert members < total < members + 2048 * 64 + 64 * 1024


@pytest.mark.parametrize("case,status", [
    ("rank49", c.UNSUPPORTED), ("fp64", c.UNSUPPORTED), ("fp32", c.UNSUPPORTED),
    ("explicit", c.UNSUPPORTED), ("n_too_large", c.UNSUPPORTED),
    ("J_r_too_large", c.UNSUPPORTED),
])
def test_batch_create_rejects_unsupported_members_without_gpu(case, status):
    d = _bf16_desc()
    good = c.make_inputs(K=256, UK=256, dK=256, obs_ptr=256, obs_i=256, obs_j=256, A=256, B=256)
    inp = good
    if case == "rank49":
        d.r = 49
    elif case == "fp64":
        d.precision = c.FP64
    elif case == "fp32":
        d.precision = c.MIXED_FP32
    elif case == "explicit":
        inp = c.make_inputs(K=256, UK=256, dK=256, obs_ptr=256, Zhat=256, V=256)
        d.gamma = 1.0
    elif case == "n_too_large":
        d.n, d.q = 70000, 70000
    elif case == "J_r_too_large":  # B must fit the gather's LDS copy: J r <= 8192
        d.r, d.J = 48, 171
    descs = [_bf16_desc(), d]
    inputs = [good, inp]
    nbytes = c.cphifi_batch_workspace_bytes(descs)
    with pytest.raises(c.CphifiError) as ei:  # fails validation before any device call
        c.cphifi_batch_create(descs, inputs, 1 << 20, nbytes, 0)
    assert ei.value.status == status
    assert "member 1" in c.last_error()


@pytest.mark.parametrize("count", [0, 257])
def test_batch_count_is_bounded(count):
    with pytest.raises(c.CphifiError) as ei:
        c.cphifi_batch_workspace_bytes([_bf16_desc()] * count)
    assert ei.value.status == c.INVALID_ARG


def _parse_table(path):
    rules = []
    for line in open(path):
        if line.startswith("#"):
            continue
        tag, trans, r_lo, r_hi, n_lo, n_hi, mw, s, ks = line.split()
        rules.append((tag, int(trans), int(r_lo), int(r_hi), int(n_lo), int(n_hi), int(mw),
                      int(s), int(ks)))
    return rules


@pytest.mark.parametrize("krange,mw", [(1024, 2), (2048, 4), (4096, 4)])
def test_batch_tile_table_is_complete_and_valid(tmp_path, krange, mw):
    """The batch autotuner's table: for each product kind, bins that tile
    1..n_max without gaps, tiles the library accepts, split-K depth in 1..16
    and about n / krange."""
    from paper_2603_25691_amd import tune

    path = tmp_path / "t.txt"
    tune._batch_table(str(path), krange, mw, 8192)
    rules = _parse_table(path)
    elts = {"bf16": c.ELT_BF16, "f64": c.ELT_F64}
    kinds = sorted({(r[0], r[1]) for r in rules})
    assert kinds == [("bf16", 0), ("f64", 0), ("f64", 1)]
    for kind in kinds:
        rs = [r for r in rules if (r[0], r[1]) == kind]
        assert rs[0][4] == 1 and rs[-1][5] >= 8192
        for a, b in zip(rs, rs[1:]):
            assert b[4] == a[5] + 1
        for tag, trans, r_lo, r_hi, n_lo, n_hi, tmw, s, ks in rs:
            assert (r_lo, r_hi) == (1, 64)
            assert c.cphifi_product_tile_ok(elts[tag], tmw, s)
            assert 1 <= ks <= 16
            mid = (n_lo + n_hi) / 2
            assert ks == max(1, min(16, round(mid / krange)))
        if kind[0] == "bf16":
            assert all(r[6] == mw for r in rs)


def test_bf16_tile_layout_follows_the_header_formula():
    # element (i, k) of a row-major bf16 matrix lands at
    # ((i / 16) (ld / 64) + k / 64) 1024 + (i % 16) 64 + k % 64 of the tiled copy
    torch = pytest.importorskip("torch")
    from paper_2603_25691_amd.torch_api import bf16_tiles
    n, ld = 37, 128
    vals = torch.arange(n * ld, dtype=torch.float32).remainder(251) + 1
    Ub = vals.view(n, ld).to(torch.bfloat16)
    T = bf16_tiles(Ub)
    assert T.shape == (48, ld) and T.stride(0) == ld
    flat = T.reshape(-1)
    for i in range(n):
        for k in range(ld):
            off = ((i // 16) * (ld // 64) + k // 64) * 1024 + (i % 16) * 64 + k % 64
            assert flat[off] == Ub[i, k]
    assert int(flat.count_nonzero()) == n * ld  # the padding rows are zero
    with pytest.raises(ValueError):
        bf16_tiles(torch.zeros(4, 40, dtype=torch.bfloat16))


def test_tiled_bf16_product_shares_tiles_and_workspace_with_row_major():
    for mw, s in [(1, 4), (2, 2), (2, 4), (4, 2), (4, 4), (1, 8)]:
        assert c.cphifi_product_tile_ok(c.ELT_BF16_TILED, mw, s) == \
            c.cphifi_product_tile_ok(c.ELT_BF16, mw, s)
    assert not c.cphifi_product_tile_ok(4, 4, 2)
    for n, r in [(100, 5), (30658, 40)]:
        assert c.cphifi_product_workspace_bytes(n, r, c.ELT_BF16_TILED) == \
            c.cphifi_product_workspace_bytes(n, r, c.ELT_BF16)
