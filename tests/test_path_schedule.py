"""CPU model of the paired path pass's schedule (no GPU).

The path kernel walks each line of a direction r with one wave and the same
line backwards (-r) with a partner wave.  Both run T = n + delta steps (T a
multiple of the chunk length K): the forward wave's extra steps come after
its line, the reverse wave's before it.  Each wave writes its own value for
its first split steps (split a multiple of K), meets the partner at a
barrier, and for the rest adds the value the partner left at that pixel.
Diagonal lines are W "wrapped" lines of one pixel per row that restart when
they cross the border.  Volume positions travel as 32-bit element offsets
advanced by a uniform stride (with a second stride at a wrap); steps outside
the line carry the no-write bit.

This model restates that arithmetic and checks, for many sizes, chunk
lengths and all four direction pairs:
  * each wave's steps visit exactly its line's pixels, in its direction's
    order, with a restart flag exactly where p - r leaves the image;
  * the two write phases partition the line, and every pixel a wave
    completes was written by the partner before the barrier;
  * every written offset lies inside the volume; the others are no-writes.
"""
import pytest

KNOWRITE = 0x80000000
DIRS = [(1, 0), (0, 1), (1, 1), (-1, 1)]        # LR, TB, TLBR, TRBL (and their reverses)


def schedule(n, K):
    delta = (K - n % K) % K
    T = n + delta
    split_fwd = K * (T // (2 * K))
    return T, delta, split_fwd, T - split_fwd


def walk(q, W, H, D, lc, fwd, K):
    """[(offset, restart, pixel index t or None)] per step of one wave."""
    dx, dy = DIRS[q]
    kind = 0 if q == 0 else (1 if q == 1 else 2)
    n = W if kind == 0 else H
    T, delta, _, _ = schedule(n, K)
    dlt = 0 if fwd else delta
    sdx, sdy = (dx, dy) if fwd else (-dx, -dy)
    if kind == 0:
        y0, x0 = lc, (0 if sdx > 0 else W - 1)
    elif kind == 1:
        x0, y0 = lc, (0 if sdy > 0 else H - 1)
    else:
        y0 = 0 if sdy > 0 else H - 1
        if fwd:
            e = lc
        else:
            v = lc + dx * (H - 1)
            e = (abs(v) % W) * (1 if v >= 0 else -1)      # C remainder keeps the sign
        x0 = e + W if e < 0 else e
    t = -dlt
    off = (y0 * W + x0) * D & 0xFFFFFFFF
    x = x0
    wrapped = False
    stride = (sdy * W + sdx) * D
    stride_wrap = (sdy * W + sdx - sdx * W) * D
    last_x = W - 1 if sdx > 0 else 0
    restart_x = 0 if sdx > 0 else W - 1
    nchunks = T // K
    c_last_checked = nchunks - 1 if (fwd and delta > 0) else -1
    out = []
    for s in range(T):
        c = s // K
        checked = c == 0 or c == c_last_checked
        if checked and (t < 0 or t >= n):
            out.append((KNOWRITE, False, None))
        else:
            assert 0 <= t < n, "an unchecked step left its line"
            rst = False
            if kind == 2:
                rst = wrapped
                wrapped = x == last_x
                cur = off
                off = (off + (stride_wrap if wrapped else stride)) & 0xFFFFFFFF
                x = restart_x if wrapped else x + sdx
            else:
                cur = off
                off = (off + stride) & 0xFFFFFFFF
            if checked and t == 0 and dlt > 0:
                rst = True            # the reverse wave's first pixel after its extra steps
            out.append((cur, rst, t))
        t += 1
    return out


def check_pair(W, H, D, Kh, Ko, q):
    dx, dy = DIRS[q]
    kind = 0 if q == 0 else (1 if q == 1 else 2)
    n = W if kind == 0 else H
    K = Kh if kind == 0 else Ko
    nlines = H if q == 0 else W
    vol = W * H * D
    T, delta, sf, sr = schedule(n, K)
    assert sf % K == 0 and sr % K == 0 and T % K == 0
    for lc in range(nlines):
        fw = walk(q, W, H, D, lc, True, K)
        rv = walk(q, W, H, D, lc, False, K)

        def pixels(seq):
            return [(((o // D) % W, (o // D) // W), r) for (o, r, _) in seq if o != KNOWRITE]

        pf, pr = pixels(fw), pixels(rv)
        assert len(pf) == n and len(pr) == n
        for seq, (sdx, sdy) in ((pf, (dx, dy)), (pr, (-dx, -dy))):
            for i, ((x, y), rst) in enumerate(seq):
                assert 0 <= x < W and 0 <= y < H
                px, py = x - sdx, y - sdy
                outside = not (0 <= px < W and 0 <= py < H)
                if i == 0:
                    assert outside, "a line starts inside the image"
                    continue
                assert rst == outside, f"restart flag wrong at step {i} of line {lc}"
                if not outside:
                    assert seq[i - 1][0] == (px, py), "not a path step"
        assert [p for p, _ in pr] == [p for p, _ in pf][::-1], "reverse wave not the same line"
        wf = {fw[s][0] for s in range(sf) if fw[s][0] != KNOWRITE}
        wr = {rv[s][0] for s in range(sr) if rv[s][0] != KNOWRITE}
        allp = {o for o, _, _ in fw if o != KNOWRITE}
        assert wf.isdisjoint(wr) and wf | wr == allp, "write phases do not partition the line"
        rf = {fw[s][0] for s in range(sf, T) if fw[s][0] != KNOWRITE}
        rr = {rv[s][0] for s in range(sr, T) if rv[s][0] != KNOWRITE}
        assert rf == wr and rr == wf, "a completed pixel was not written by the partner"
        assert all(o + D <= vol for o in allp)


@pytest.mark.parametrize("W,H", [(1, 1), (2, 1), (1, 2), (3, 5), (7, 3), (64, 48), (65, 33),
                                 (97, 33), (321, 17), (30, 70), (9, 100), (17, 257)])
@pytest.mark.parametrize("Kh,Ko", [(32, 8), (16, 16), (32, 16)])
def test_pair_schedule(W, H, Kh, Ko):
    for q in range(4):
        check_pair(W, H, 2, Kh, Ko, q)


def test_pair_schedule_benchmark_frame():
    """The 1242x375 frame, every pair, the product's chunk lengths."""
    for q in range(4):
        check_pair(1242, 375, 2, 32, 8, q)
