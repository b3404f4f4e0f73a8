"""CPU replay of the shifted-solve kernels' index arithmetic for every shape
of the batched ensemble, the serving stream and the full-size workloads:
every global row a thread reads or writes lies in [0, n), every LDS entry it
touches lies inside its staging area, and every partial-sum row lies inside
the buffer the plan allocates.

A batched ensemble solve once faulted the GPU with an illegal address: the
paired real shifts k = 0 and k = ell/2 (one work item) read the neighbour
rows s0 - 1 and s0 + MR of a thread's chunk without clamping, and threads
whose chunk starts past the end of the system (s0 > n, present whenever
P * MR exceeds n by more than one chunk) read before or after the array.
The kernel now clamps both; these tests keep that and every other access of
the tridiag_pipe_body / tridiag_uniform_body expressions (csrc/tridiag.hip)
in range.  The expressions below restate the kernel's, statement by
statement."""
import numpy as np
import pytest

from paper_2304_12597_amd import workloads as wl

CUS = 256


def choose_tri(n, prec):
    """pd_choose_tri: rows per thread MR and threads per system P (the
    smallest power of two with P MR >= n)."""
    MR = 8
    if n > 8192:
        MR = 16
    if prec == 0 and n > 4096:
        MR = 16
    if n <= 64:
        MR = 4
    P = 1
    while P * MR < n:
        P *= 2
    BT = 512 if prec == 0 else 1024
    spb = BT // P if P >= 16 else 64
    spb = max(spb, 1)
    pipe = prec == 0 and P >= 64
    return MR, P, spb, pipe


def lg_of(MR):
    return 0 if MR == 16 else (1 if MR == 8 else 2)


def pipe_entry(lt, q, MR):
    return lt * MR + ((q + (lt >> lg_of(MR))) & (MR - 1))


def check_pipe(n, F2):
    """tridiag_pipe_body (complex128, P >= 64) for one problem."""
    MR, P, spb, pipe = choose_tri(n, 0)
    assert pipe
    rows = P * MR
    lt = np.arange(P)
    s0 = lt * MR
    ln = np.clip(n - s0, 0, MR)
    lane = lt & 63
    wib = lt >> 6
    LG = lg_of(MR)
    # issue(): one DMA window of 16 staging entries per instruction
    for wdw in range(4 * MR):
        e0 = wib * 64 * MR + wdw * 16
        e = e0 + (lane >> 2)
        tl = e // MR
        j = e & (MR - 1)
        q = (j - (tl >> LG)) & (MR - 1)
        r = np.minimum(tl * MR + q, n - 1)
        assert r.min() >= 0 and r.max() < n
        assert e0.min() >= 0 and (e0 + 15).max() < rows           # LDS window
        # the staged entry e holds row tl*MR + q: the rotation is a bijection
        assert np.all(pipe_entry(tl, q, MR) == e)
    # work(), paired real shifts: rows of the thread's chunk and neighbours
    for q in range(MR):
        r = np.minimum(s0 + q, n - 1)
        assert r.min() >= 0 and r.max() < n
    rl = np.where((lt > 0) & (s0 - 1 < n), s0 - 1, 0)
    rr = np.where(s0 + MR < n, s0 + MR, n - 1)
    assert rl.min() >= 0 and rl.max() < n and rr.min() >= 0 and rr.max() < n
    # work(), complex shifts: staging entries of the chunk and neighbours
    for q in range(MR):
        assert pipe_entry(lt, q, MR).max() < rows
    assert pipe_entry(np.maximum(lt - 1, 0), MR - 1, MR).max() < rows
    assert pipe_entry(np.where(lt + 1 < P, lt + 1, lt), 0, MR).max() < rows
    # mode 1 stores after the 4x4 lane-quad transpose: row < n is tested
    c = lt & 3
    qb = lt & ~3
    hits = np.zeros(n, dtype=np.int64)
    for q in range(MR):
        row = (qb + (q & 3)) * MR + (q & ~3) + c
        assert row.min() >= 0
        hits += np.bincount(row[row < n], minlength=n)
    assert np.all(hits == 1)                        # every row written exactly once
    # one-time staging of x / M v with a zero halo (pad16 layout, count = rows + 2)
    count = rows + 2
    pad16 = lambda i: i + (i >> 4)
    assert pad16(count - 1) < 2 * rows              # fits the complex128 area
    # partial sums: one row per block, blocks = min(items, CUs)
    nitems = F2 - 1
    G = min(nitems, CUS)
    assert G <= min(nitems, CUS)


def check_uniform(n, prec):
    """tridiag_uniform_body (complex64 plans and P < 64)."""
    MR, P, spb, _ = choose_tri(n, prec)
    rows = P * MR
    sstride = rows + 2
    lt = np.arange(P)
    s0 = lt * MR
    # stage_halo: idx - 1 clamped to [0, n) for idx < count
    for b in range(0, sstride, P):
        idx = b + lt
        i = idx - 1
        ic = np.clip(i, 0, n - 1)
        assert ic.min() >= 0 and ic.max() < n
    # the DMA path of complex128 systems with P >= 64
    if prec == 0 and P >= 64:
        wb = lt & ~63
        for q in range(MR):
            i0 = q * P + wb
            i = np.minimum(i0 + (lt & 63), n - 1)
            assert i.min() >= 0 and i.max() < n
            assert (1 + i0 + 63).max() <= sstride - 1
    # right-hand side reads stage[i], stage[i + 1], stage[i + 2] for rows < n
    for q in range(MR):
        i = s0 + q
        ok = i < n
        assert (i[ok] + 2).max(initial=0) < sstride


def ensemble_shapes():
    return sorted({(n, ell) for n, ell, _ in wl.ensemble_params(count=512)})


def check_shape(n, ell, prec):
    MR, P, spb, pipe = choose_tri(n, prec)
    if pipe:
        check_pipe(n, ell // 2 + 1)
    else:
        check_uniform(n, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_ensemble_shapes_in_range(prec):
    # the index arithmetic depends on n (ell only sets the number of items)
    for n in sorted({n for n, _ in ensemble_shapes()}):
        check_shape(n, 64, prec)


def test_serving_and_headline_shapes_in_range():
    shapes = {(8191, 2048), (63, 32), (8192, 4096), (2, 2), (3, 4), (65, 8), (4097, 16)}
    for r in wl.serving_stream(count=256, rate=1.0, build=False):
        p = r.problem
        if p.dims == 1:
            shapes.add((p.n, p.ell))
    for n in sorted({n for n, _ in shapes}):
        for prec in (0, 1):
            if prec == 0 and n > 8192:
                continue
            check_shape(n, 64, prec)


def test_unclamped_neighbour_read_is_caught():
    """The check above rejects the pre-fix neighbour rows (s0 - 1 and s0 + MR
    without clamping) on an ensemble shape where chunks start past n."""
    n = 2049                    # P = 512 rows / MR = 8: chunks 257.. start past n
    MR, P, spb, pipe = choose_tri(n, 0)
    lt = np.arange(P)
    s0 = lt * MR
    assert (s0 > n).any()
    bad_right = s0 + MR
    assert bad_right.max() >= n
