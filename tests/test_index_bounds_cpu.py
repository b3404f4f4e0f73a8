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
That pair is now staged through LDS like every other slot; these tests keep
every access of the tridiag_pipe_body / tridiag_uniform_body expressions
(csrc/tridiag.hip) in range.  The expressions below restate the kernel's, statement by
statement."""
import numpy as np
import pytest

from paper_2304_12597_amd import workloads as wl

CUS = 256
MAX_LDS = 160 * 1024


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
    # issue(), complex slots: one 16-byte DMA window of 64 entries per instruction
    seen = np.zeros(rows, dtype=np.int64)
    for wdw in range(MR):
        e0 = wib * 64 * MR + wdw * 64
        e = e0 + lane
        tl = e // MR
        j = e & (MR - 1)
        q = (j - (tl >> LG)) & (MR - 1)
        r = np.minimum(tl * MR + q, n - 1)
        assert r.min() >= 0 and r.max() < n
        assert e0.min() >= 0 and (e0 + 63).max() < rows           # LDS window
        assert np.all(e0 == (e0 // 64) * 64) and np.all(e0 == e - lane)   # 64 entries per wave
        assert np.all(pipe_entry(tl, q, MR) == e)
        seen += np.bincount(e, minlength=rows)
    assert np.all(seen == 1)                        # every staging entry filled once
    # issue(), paired real shifts: one 4-byte DMA window of 16 entries per instruction
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
        # paired real shifts (slot 0): lanes with bit 1 read the real part of
        # frequency ell/2, the others that of frequency 0; dword lane & 1 of the row
        src_row = np.where(lane & 2, F2 - 1, 0)
        dw = r * 4 + (lane & 1)
        assert src_row.max() < F2 and dw.max() < 4 * n and np.all((dw & 3) < 2)
        # the four lanes of an entry fill dwords 0, 1 (k = 0) and 2, 3 (k = ell/2)
        assert np.all(np.where(lane & 2, 2, 0) + (lane & 1) == (lane & 3))
    # work(): staging entries of the chunk and neighbours (every slot)
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
    # mode 1: -w M x from direct loads of x_{s0-1} .. x_{s0+MR}, clamped
    for j in range(MR + 2):
        i = s0 - 1 + j
        ic = np.where(i < 0, 0, np.where(i < n, i, n - 1))
        assert ic.min() >= 0 and ic.max() < n
    # mode 2: one-time staging of M v with a zero halo (pad16 layout, count = rows + 2)
    count = rows + 2
    pad16 = lambda i: i + (i >> 4)
    assert pad16(count - 1) < 2 * rows              # fits the complex128 area
    # partial sums: one row per block, blocks = min(items, CUs)
    nitems = F2 - 1
    G = min(nitems, CUS)
    assert G <= min(nitems, CUS)
    # LDS: stage | P Row3 exchange entries per group | two factor buffers,
    # within the 160 KiB of a CU
    nfp = (6 * (MR - 1) + 63) // 64 * 64
    lds = spb * (rows + 3 * P + 2 * nfp) * 16
    assert lds <= MAX_LDS, (n, lds)
    # recurrence form (pd_scan.h): the issue split into four parts covers
    # each window once; the constants' one 64-entry DMA window (wave 0)
    # reads entries min(idx, NF - 1) of row F2 or k < F2 of the (F2 + 1) x NF
    # table and fills entries 0..63 of a factor buffer of nfp >= 64 entries;
    # the solve reads entries 0..8 + MR of it; the exchange area xw holds
    # 3 * (P / 64) complex128 entries inside the group's P Row3 entries
    NF = 6 * (MR - 1)
    parts = [w for part in range(4) for w in range(part * (MR // 4), (part + 1) * (MR // 4))]
    assert sorted(parts) == list(range(MR))
    idx = np.minimum(np.arange(64), NF - 1)
    assert idx.max() < NF and nfp >= 64 and 8 + MR < NF
    assert 3 * (P // 64) * 16 <= P * 48


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


def pipe_schedule(nitems, nblk, spb, MR):
    """The item loop of tridiag_pipe_body, restated: per block, the sequence
    of DMA issues (slot, factor buffer) and solves (slot, factor buffer, ops).
    At 16 rows per thread block 0 runs the paired slot 0 before its regular
    items (factor buffer 1); otherwise slot 0 is an ordinary item of the
    loop."""
    pair_first = MR == 16
    out = []
    for blk in range(nblk):
        ev = []
        item, buf = blk, 0
        if pair_first and blk == 0:
            ev.append(("issue", 0, 1))
            ev.append(("solve", 0, 1, "dual"))
            if nblk < nitems:
                ev.append(("issue", nblk, 0))
            item = nblk
        elif blk < nitems:
            ev.append(("issue", item * spb, 0))
        while item < nitems:
            slot = item * spb
            ops = "dual" if (not pair_first and slot == 0) else "cplx"
            ev.append(("solve", slot, buf, ops))
            if item + nblk < nitems:
                ev.append(("issue", (item + nblk) * spb, buf ^ 1))
            item += nblk
            buf ^= 1
        out.append(ev)
    return out


@pytest.mark.parametrize("MR", [8, 16])
@pytest.mark.parametrize("nitems,nblk", [(1024, 256), (1023, 256), (256, 256), (5, 5),
                                         (64, 37), (1, 1), (2, 2), (3, 2)])
def test_pipe_item_schedule(MR, nitems, nblk):
    """Every slot is solved once, with the factor buffer its DMA filled, the
    paired slot 0 with the componentwise (dual) arithmetic; an item's
    successor streams into the other factor buffer, and the right-hand-side
    staging area is refilled only after the item that read it."""
    spb = 1
    solved = []
    for ev in pipe_schedule(nitems, nblk, spb, MR):
        pending = None            # (slot, buffer) of the DMA in flight
        in_use = None             # factor buffer of the item being solved
        for e in ev:
            if e[0] == "issue":
                assert pending is None      # one staging area: consumed first
                assert e[2] != in_use       # factors of the solve in progress kept
                pending = (e[1], e[2])
            else:
                _, slot, buf, ops = e
                assert pending == (slot, buf)
                assert (ops == "dual") == (slot == 0)
                pending = None
                in_use = buf
                solved.append(slot)
        assert pending is None
    assert sorted(solved) == list(range(nitems * spb))


# ------------------------------------------- chunked capacitance product --

def cp_chunking(n):
    """pd_cp_chunking: nc <= 64 chunks of m rows (m odd, >= 3), the last one
    2..m+1 rows."""
    m = max(3, (n + 63) // 64)
    if m % 2 == 0:
        m += 1
    nc = (n + m - 1) // m
    L = n - (nc - 1) * m
    if L == 1 and nc > 1:
        nc -= 1
        L = m + 1
    return m, nc, L


CP_SPLITS, CP_KW, CP_VW, CP_UW, CP_PF, CP1_WAVES = 16, 4, 2, 66, 36, 5


def cp_layout(n, F2, ell=None):
    """pd_cp_layout and the pairing choice of pd_cp_tables (csrc/capprod.hip):
    launch shapes and table sizes."""
    m, nc, L = cp_chunking(n)
    c = dict(m=m, nc=nc, L=L, N0=m - 1, NL=L - 1)
    c["Q"] = (c["N0"] + 2 + 3) // 4
    c["NT"] = (nc + 15) // 16
    c["NTc"] = 16 * c["NT"]
    c["NH"] = c["NT"] // 2 if c["NT"] % 2 == 0 else c["NT"]
    c["VL"] = (max(n + 3, (c["NTc"] - 1) * m + 4 * c["Q"] + 2) + 1) & ~1
    c["G1"] = (F2 + 3) // 4
    ell = 2 * (F2 - 1) if ell is None else ell
    c["pair"] = ell % 2 == 0 and F2 >= 5 and (F2 - 1) % 4 == 0
    c["G1run"] = (F2 - 1) // 4 if c["pair"] else c["G1"]
    c["MT"] = (c["N0"] + 15) // 16
    c["Sk"] = CP_SPLITS - 1
    c["KPS"] = (F2 + c["Sk"] - 1) // c["Sk"]
    c["KPT"] = max(4 * c["G1"], c["Sk"] * c["KPS"])
    c["HLS"] = c["NL"] + 2
    c["NV"] = c["NL"] + nc
    c["sizes"] = dict(T1=c["G1"] * c["Q"] * 64, hL=4 * c["G1"] * c["HLS"], red=8 * F2,
                      gk=c["KPT"], T3=c["MT"] * c["KPT"] * 64, c1=c["KPT"] * c["NL"],
                      T4=c["MT"] * c["Q"] * 64, L1h=c["NL"] * (c["NL"] + 2),
                      U=c["KPT"] * CP_UW, tiles=CP_SPLITS * c["MT"] * 16 * c["NTc"],
                      vrow=CP_SPLITS * c["NV"])
    return c


def cp_sidx(t, gq, Q):
    """cp_sidx: window index of matrix-core step t for lane group gq."""
    B16 = Q >> 4
    t = np.asarray(t)
    R = Q - (B16 << 4)
    full = ((t >> 4) << 6) + (gq << 4) + (t & 15)
    part = (B16 << 6) + R * gq + (t - (B16 << 4))
    return np.where(t < (B16 << 4), full, part)


def check_cp(n, F2, max_lds=160 * 1024):
    """cp_freq_kernel / cp_out_kernel / cp_sum_kernel (csrc/capprod.hip):
    every LDS, table, workspace and output index is in range, the window and
    frequency contractions cover what they must, and the sum launch writes
    every output row exactly once.  False when the plan would not use them."""
    c = cp_layout(n, F2)
    m, nc, L, N0, NL = c["m"], c["nc"], c["L"], c["N0"], c["NL"]
    Q, NT, NTc, NH, VL = c["Q"], c["NT"], c["NTc"], c["NH"], c["VL"]
    MT, Sk, KPS, KPT, NV = c["MT"], c["Sk"], c["KPS"], c["KPT"], c["NV"]
    sz = c["sizes"]
    assert m % 2 == 1 and 1 <= nc <= 64 and 2 <= L <= m + 1 and (nc - 1) * m + L == n
    assert 4 * Q >= N0 + 2 and NTc >= nc and NTc <= 64 and 16 * MT >= N0
    lds1 = (VL + CP1_WAVES * 64 * 4) * 8
    lds2 = VL * 8 + (CP_KW - 1) * 2 * 64 * 32
    if lds1 > max_lds or lds2 > max_lds:
        return False            # pd_cp_fits: the plan takes the per-frequency path
    lane = np.arange(64)
    gq, cl = lane >> 4, lane & 15
    # the window mapping is a bijection onto [0, 4Q)
    s_all = np.concatenate([cp_sidx(np.arange(Q), g, Q) for g in range(4)])
    assert np.array_equal(np.sort(s_all), np.arange(4 * Q))
    # v staging, both alignments: vs[o + i] = v[i], pairs at vs[2 + 2p],
    # zeros in [0, o) and [o + n, VL); every entry written once
    for sh in (0, 1):
        o = 2 - sh
        npairs = (n - sh) // 2
        w = np.zeros(VL, dtype=np.int64)
        p = np.arange(npairs)
        assert (sh + 2 * p + 1).max(initial=0) < n
        np.add.at(w, 2 + 2 * p, 1)
        np.add.at(w, 3 + 2 * p, 1)
        if sh:
            w[o] += 1
        if (n - sh) & 1:
            w[o + n - 1] += 1
        w[:o] += 1
        w[o + n:] += 1
        assert (w == 1).all() and o + n <= VL
        # windows (o - 1 + c m + s, s < 4Q) and the reduced system's rows
        col = np.arange(NTc)
        assert (o - 1 + col.max() * m + 4 * Q - 1) < VL
        assert (o - 1 + (nc - 1) * m + NL + 1) < VL
        lc = np.minimum(lane, nc - 1)
        i = np.where(lc == nc - 1, n - 1, lc * m + N0)
        assert (o + i - 1).min() >= 0 and (o + i + 1).max() < VL and (i[:nc] < n).all()
    # ---- launch 1 (G1run blocks x 5 waves) ----
    pair, G1run = c["pair"], c["G1run"]
    Fs = F2 - 1 if pair else F2
    kseen = np.zeros(F2, dtype=np.int64)
    for blk in range(G1run):
        for wave in range(CP1_WAVES):
            if wave < 4:
                kw = 4 * blk + wave if 4 * blk + wave < Fs else -1
            else:
                kw = F2 - 1 if (pair and blk == 0) else -1
            if kw >= 0:
                kseen[kw] += 1
            kq = kw if kw >= 0 else 4 * blk
            assert 0 <= kq < F2 and kq * 8 + 7 < sz["red"]
            assert (kq * c["HLS"] + NL + 1) < sz["hL"]
            if kw >= 0:
                assert kw * CP_UW + CP_UW - 1 < sz["U"]
        assert (blk * Q + Q - 1) * 64 + 63 < sz["T1"]
        # Ex: [CP1_WAVES][64][4] after vs
        assert ((CP1_WAVES - 1) * 64 + 63) * 4 + 3 < CP1_WAVES * 64 * 4
    assert (kseen == 1).all()                  # every frequency once
    if pair:
        assert 4 * G1run + 1 == F2 and G1run <= c["G1"]
    # ---- launch 2 (MT x S x NH blocks) ----
    for local in (0, 1):
        S = Sk + local
        TPB = NT // NH
        nmw = TPB * CP_KW
        assert nmw + CP_VW <= 2 * CP_KW + CP_VW and TPB * NH == NT and TPB <= 2
        assert Sk * KPS >= F2 and KPT >= Sk * KPS and KPT >= 4 * c["G1"]
        grid = MT * S * NH
        blocks = {(b % NH, (b // NH) % MT, b // (NH * MT)) for b in range(grid)}
        assert len(blocks) == grid
        qs = (KPS + CP_KW - 1) // CP_KW
        for sp in sorted({0, Sk - 1}):
            covered = []
            for kh in range(CP_KW):
                kb = min(kh * qs, KPS)
                ke = min(kb + qs, KPS)
                ka = sp * KPS + kb
                cnt = ke - kb
                covered += list(range(ka, ka + cnt))
                if cnt == 0:
                    continue
                assert ka + cnt <= (sp + 1) * KPS <= KPT
                assert ((MT - 1) * KPT + ka + cnt - 1) * 64 + 63 < sz["T3"]
                for nh in range(NH):
                    for tl in range(TPB):
                        col = (nh * TPB + tl) * 16 + cl
                        pb = ((ka + cnt - 1) * CP_UW + col + (gq >> 1)) * 2 + (gq & 1)
                        assert pb.max() < 2 * sz["U"] and col.max() + 1 < CP_UW
            # the quarters cover the split's frequencies once
            assert covered == list(range(sp * KPS, sp * KPS + KPS))
            # vector rows: each rho < NV once per split over its MT NH blocks
            NB = MT * NH
            seen = np.zeros(NV, dtype=np.int64)
            for b in range(NB):
                j0 = 0
                while b + j0 * NB < NV:
                    for vw in range(CP_VW):
                        rho = b + (j0 + 4 * vw + (lane >> 4)) * NB
                        ok = (rho < NV) & ((lane & 15) == 0)
                        np.add.at(seen, rho[ok], 1)
                    j0 += 4 * CP_VW
            assert (seen == 1).all()
            kg = np.arange(16)
            nit = (KPS - kg + 15) >> 4          # groups with nit = 0 load nothing
            kmax = (sp * KPS + kg + 16 * (nit - 1))[nit > 0]
            assert kmax.max() < KPT
            assert ((kmax.max() * NL + NL - 1) < sz["c1"]) and kmax.max() * CP_UW + nc < sz["U"]
            assert kmax.max() < sz["gk"]
            ks = np.sort(np.concatenate([sp * KPS + g + 16 * np.arange(nit[g]) for g in kg]))
            assert np.array_equal(ks, np.arange(sp * KPS, sp * KPS + KPS))
        if local:
            assert ((MT - 1) * Q + Q - 1) * 64 + 63 < sz["T4"]
            assert (NL - 1) * (NL + 2) + NL + 1 < sz["L1h"] or NL == 0
        assert ((CP_KW - 2) * TPB + TPB - 1) * 64 + 63 < (CP_KW - 1) * 2 * 64
        # ---- launch 3: every output row exactly once ----
        hits = np.zeros(n, dtype=np.int64)
        nt = MT * 16 * NTc
        it = np.arange(nt)
        mt_, e = it // (16 * NTc), it % (16 * NTc)
        r_, c_ = e // NTc, e % NTc
        s_ = 16 * mt_ + r_
        ok = (c_ < nc - 1) & (s_ < N0)
        np.add.at(hits, (c_ * m + s_)[ok], 1)
        assert ((S - 1) * nt + it.max()) < sz["tiles"]
        rho = np.arange(NV)
        i = np.where(rho < NL, (nc - 1) * m + rho,
                     np.where(rho - NL == nc - 1, n - 1, (rho - NL) * m + N0))
        assert i.min() >= 0 and i.max() < n
        np.add.at(hits, i, 1)
        assert ((S - 1) * NV + NV - 1) < sz["vrow"]
        assert (hits == 1).all()
    return True


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 63, 64, 65, 127, 128, 129, 130, 255, 1000,
                               4095, 4097, 8191, 8192, 12759, 16383, 16384, 18000, 20000])
def test_chunked_capacitance_indices(n):
    for ell in (2, 16, 2048):
        check_cp(n, ell // 2 + 1)


def test_chunked_capacitance_headline_fits():
    # the 1D FEM workload of the headline (n = 8191, ell = 2048) runs on it
    assert check_cp(8191, 1025)


def test_chunked_capacitance_ensemble_shapes():
    for n in sorted({n for n, _ in ensemble_shapes()}):
        check_cp(n, 33)
