"""CPU model of the stream-K work assignment of the n x n by n x r products
(the FP64 transposed form and the tiled BF16 form, gemm.hip).

W workgroups share the T = (row blocks) x (k chunks) iterations, workgroup w
taking [w T / W, (w + 1) T / W); a workgroup walks its range row block by row
block and writes one partial slab per row block it touches (slab index = w
minus the first contributor of that row block); the last contributor of a row
block zeroes the slabs no contributor writes, so every row sums the plan's
`ksplit` slabs.  The model replays the kernels' index arithmetic and the
plan's choice of ksplit with Python integers and checks, for many n:

* every (row block, chunk) is multiplied exactly once, with its k range
  chunk-aligned inside [0, n);
* every slab index is below the plan's ksplit, and every (row block, slab) is
  either written by exactly one contributor or zeroed, never both.
"""

import pytest


def sk_first(x, wgs, t):
    # the workgroup whose range holds iteration x
    return ((x + 1) * wgs - 1) // t


def plan_slabs(nrb, nch, w):
    t = nrb * nch
    ksp = 1
    for b in range(nrb):
        ksp = max(ksp, sk_first((b + 1) * nch - 1, w, t) - sk_first(b * nch, w, t) + 1)
    return ksp


def replay(n, rows, bk, w):
    nrb = (n + rows - 1) // rows
    nch = (n + bk - 1) // bk
    t = nrb * nch
    ksp = plan_slabs(nrb, nch, w)
    done, written, zeroed = set(), set(), set()
    for wg in range(w):
        c, c1 = wg * t // w, (wg + 1) * t // w
        while c < c1:
            b = c // nch
            cend = min(c1, (b + 1) * nch)
            wf, wl = sk_first(b * nch, w, t), sk_first((b + 1) * nch - 1, w, t)
            slab = wg - wf
            assert 0 <= slab < ksp
            if wg == wl:
                zeroed.update((b, s) for s in range(wl - wf + 1, ksp))
            kbeg, kend = (c - b * nch) * bk, min(n, (cend - b * nch) * bk)
            assert kbeg % bk == 0 and 0 <= kbeg < kend <= n
            for j in range(c - b * nch, cend - b * nch):
                assert (b, j) not in done
                done.add((b, j))
            assert (b, slab) not in written
            written.add((b, slab))
            c = cend
    assert len(done) == t
    for b in range(nrb):
        for s in range(ksp):
            assert ((b, s) in written) != ((b, s) in zeroed)
    return ksp


@pytest.mark.parametrize("n", [64, 129, 1000, 4097, 5000, 10300, 12345, 30658])
@pytest.mark.parametrize("rows,bk,w", [(256, 8, 512), (128, 16, 512), (64, 32, 512),
                                       (256, 64, 256)])
def test_stream_k_assignment_covers_every_chunk_once(n, rows, bk, w):
    if (n + rows - 1) // rows * ((n + bk - 1) // bk) < w:
        pytest.skip("fewer iterations than workgroups: the plans keep split-K")
    replay(n, rows, bk, w)


def test_model_catches_an_off_by_one_first_contributor():
    """A plausible slip (taking the first contributor of a row block as the
    workgroup of its first iteration minus one) breaks the slab bookkeeping."""
    def bad_first(x, wgs, t):
        return max(0, ((x + 1) * wgs - 1) // t - 1)

    global sk_first
    good = sk_first
    try:
        sk_first = bad_first
        with pytest.raises(AssertionError):
            replay(30658, 256, 64, 256)
    finally:
        sk_first = good
