"""CPU model of the chunk loops of the product tiles (gemm_tiles.h).

Each tile walks its k-range [kbeg, kend) in chunks of BK rows with operand
registers in flight ahead of the MFMAs (two buffers a0 / a1 for the FP64 and
FP32 tiles and the BF16 tile at depth 2; three for the BF16 tile at depth 3)
and the n x r operand double-buffered in LDS.  The model below replays the
same control flow (the steady state, the peeled steps, the tail-aware fetch)
with plain Python integers and checks, for every span, chunk size, split and
row count enumerated:

* every full-width fetch of the n x n operand covers rows [k0, k0 + BK) inside
  [kbeg, kend) (and so inside U's storage); only the chunk that holds the k
  tail goes through the clamped fetch, whose reads stay in [0, n);
* every chunk is fetched once and multiplied once, in order, from the register
  buffer and the LDS buffer that hold it, and an LDS buffer is overwritten only
  after the chunk it held has been multiplied.

A GPU fault once came from the steady state prefetching the partial k tail with
the full-width loader (a read of up to BK - 1 rows past the end of U); the
model reproduces that mistake when the steady-state bound is loosened (checked
below), so a regression of the bound fails here, on the CPU.
"""

import itertools

import pytest


class Trace:
    def __init__(self, n, kbeg, kend, bk):
        self.n, self.kbeg, self.kend, self.bk = n, kbeg, kend, bk
        span = kend - kbeg
        self.nfull = span // bk if span > 0 else 0
        self.has_tail = span > 0 and span % bk != 0
        self.nchunk = self.nfull + (1 if self.has_tail else 0)
        self.reg = {}         # register buffer -> chunk it holds
        self.lds = {}         # LDS buffer -> chunk it holds
        self.lds_used = {}    # LDS buffer -> whether its chunk was multiplied
        self.done = []

    def fetch_full(self, buf, c):
        k0 = self.kbeg + c * self.bk
        assert k0 >= self.kbeg and k0 + self.bk <= self.kend, ("full fetch", c, k0)
        assert k0 + self.bk <= self.n
        self.reg[buf] = c

    def fetch_tail_aware(self, buf, c):
        if c == self.nfull:  # the clamped loader: rows min(k, n - 1), zero past kend
            k0 = self.kbeg + c * self.bk
            for k in range(k0, k0 + self.bk):
                assert 0 <= min(k, self.n - 1) < self.n
            self.reg[buf] = c
        else:
            self.fetch_full(buf, c)

    def store_x(self, lbuf, c):
        if lbuf in self.lds:
            assert self.lds_used[lbuf], ("LDS buffer overwritten before use", lbuf)
        self.lds[lbuf] = c
        self.lds_used[lbuf] = False

    def compute(self, buf, lbuf, c):
        assert self.reg.get(buf) == c, ("register buffer", buf, c, self.reg)
        assert self.lds.get(lbuf) == c, ("LDS buffer", lbuf, c, self.lds)
        assert c == len(self.done), ("order", c, self.done)
        self.lds_used[lbuf] = True
        self.done.append(c)

    def finish(self):
        assert self.done == list(range(self.nchunk))


def k4_loop(t, steady_bound=2):
    """gemm_k4_tile / gemm_f64x4_tile: two register buffers."""
    if t.nchunk == 0:
        return t
    t.fetch_tail_aware(0, 0)
    t.store_x(0, 0)
    c = 0
    while c + steady_bound < t.nfull:  # chunks c + 1 and c + 2 are full ones
        t.fetch_full(1, c + 1)
        t.compute(0, c & 1, c)
        t.store_x((c + 1) & 1, c + 1)
        c += 1
        t.fetch_full(0, c + 1)
        t.compute(1, c & 1, c)
        t.store_x((c + 1) & 1, c + 1)
        c += 1
    while True:
        more = c + 1 < t.nchunk
        if more:
            t.fetch_tail_aware(1, c + 1)
        t.compute(0, c & 1, c)
        if more:
            t.store_x((c + 1) & 1, c + 1)
        if not more:
            break
        c += 1
        more = c + 1 < t.nchunk
        if more:
            t.fetch_tail_aware(0, c + 1)
        t.compute(1, c & 1, c)
        if more:
            t.store_x((c + 1) & 1, c + 1)
        if not more:
            break
        c += 1
    return t


def bf16_loop(t, depth):
    """gemm_bf16_tile: U is zero-padded past n and kper is a multiple of BK, so
    every chunk is fetched full width (reads stay below round_up(n, BK))."""
    nchunk = (t.kend - t.kbeg + t.bk - 1) // t.bk if t.kend > t.kbeg else 0
    t.nchunk, t.nfull = nchunk, nchunk

    def load(buf, c):
        k0 = t.kbeg + c * t.bk
        assert 0 <= c < nchunk and k0 + t.bk <= -(-t.n // t.bk) * t.bk
        t.reg[buf] = c

    if nchunk == 0:
        return t
    if depth == 3:
        load(0, 0)
        t.store_x(0, 0)
        if nchunk > 1:
            load(1, 1)
        c = 0
        ring = [0, 1, 2]

        def step(cur, ahead):
            nonlocal c
            load(ahead, c + 2)
            t.compute(cur, c & 1, c)
            t.store_x((c + 1) & 1, c + 1)
            c += 1

        while c + 5 <= nchunk:
            step(0, 2)
            step(1, 0)
            step(2, 1)

        def tail(cur, ahead):
            nonlocal c
            if c >= nchunk:
                return
            more = c + 1 < nchunk
            if c + 2 < nchunk:
                load(ahead, c + 2)
            t.compute(cur, c & 1, c)
            if more:
                t.store_x((c + 1) & 1, c + 1)
            c += 1

        tail(0, 2)
        tail(1, 0)
        tail(2, 1)
        tail(0, 2)
        del ring
        return t
    load(0, 0)
    t.store_x(0, 0)
    c = 0
    while c + 2 < nchunk:
        load(1, c + 1)
        t.compute(0, c & 1, c)
        t.store_x((c + 1) & 1, c + 1)
        c += 1
        load(0, c + 1)
        t.compute(1, c & 1, c)
        t.store_x((c + 1) & 1, c + 1)
        c += 1
    if c + 1 < nchunk:
        load(1, c + 1)
        t.compute(0, c & 1, c)
        t.store_x((c + 1) & 1, c + 1)
        c += 1
        t.compute(1, c & 1, c)
    else:
        t.compute(0, c & 1, c)
    return t


def splits(n, bk, ksplit):
    """The k-ranges of make_gemm_plan: kper = round_up(ceil(n / ksplit), bk)."""
    kper = -(-n // ksplit)
    kper = -(-kper // bk) * bk
    ks = -(-n // kper)
    return [(s * kper, min(n, (s + 1) * kper)) for s in range(ks)]


# FP64 / FP32 tiles: BK = 4 S with S in {2, 4, 8}; BF16: BK = 32 S, S in {2, 4}
K4_BK = (8, 16, 32)
BF16_BK = (64, 128)
NS = list(range(1, 70)) + [127, 128, 129, 255, 256, 257, 1000, 1023, 30658]


@pytest.mark.parametrize("bk", K4_BK)
def test_k4_loop_fetches_stay_in_range(bk):
    for n, ksplit in itertools.product(NS, (1, 2, 3, 4, 7, 16)):
        for kbeg, kend in splits(n, bk, ksplit):
            k4_loop(Trace(n, kbeg, kend, bk)).finish()


@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("bk", BF16_BK)
def test_bf16_loop_fetches_stay_in_range(bk, depth):
    for n, ksplit in itertools.product(NS, (1, 2, 3, 5, 16)):
        for kbeg, kend in splits(n, bk, ksplit):
            bf16_loop(Trace(n, kbeg, kend, bk), depth).finish()


def test_model_catches_full_fetch_of_the_tail():
    """The loosened steady-state bound (c + 1 < nfull) prefetches the partial
    tail chunk with the full-width loader: the model must flag it."""
    with pytest.raises(AssertionError):
        for n in NS:
            for kbeg, kend in splits(n, 8, 1):
                k4_loop(Trace(n, kbeg, kend, 8), steady_bound=1).finish()
