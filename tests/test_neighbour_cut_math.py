"""The arithmetic behind the neighbour build's row cut, checked in float32 on the
CPU (numpy rounds each float32 operation to nearest, as the GPU does).

A candidate whose staged x offset q lies below xo - reach (or above xo + reach),
with reach = sqrtf(cut_hi) (1 + 2^-12) and the bound rounded once, has
fl(ax * ax) >= cut_hi for ax = fl(xo - q): the FP32 test would reject it, so
leaving it out changes no list.  The check sweeps the extreme x offsets a block
box can hold (up to 128 cells of width w >= 2h) and the candidates closest to
the bound."""
import numpy as np

f32 = np.float32


def cut_rejects(xo, q, cut_hi):
    ax = f32(xo - q)
    return f32(ax * ax) >= cut_hi


def test_candidates_beyond_the_reach_fail_the_fp32_test():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        h = 10.0 ** rng.uniform(-4, 1)
        w = 2.0 * h * rng.uniform(1.0, 4.0 / 3.0)           # cell width >= 2h
        X = w * rng.integers(3, 129)                          # box width, cells
        cut2 = (2.0 * h) ** 2
        band = max(1e-5, 3.0 * (2.0 ** -23 * X / h + 2.0 ** -22))
        cut_hi = f32(cut2 * (1.0 + band))
        reach = f32(f32(np.sqrt(cut_hi)) * f32(1.0 + 2.0 ** -12))
        xo = f32(rng.uniform(w, X - w))                       # the particle's offset
        lo_x, hi_x = f32(xo - reach), f32(xo + reach)
        # the candidates nearest the bounds that the cut leaves out
        below = lo_x
        above = hi_x
        for _k in range(4):
            below = np.nextafter(below, f32(-np.inf), dtype=np.float32)
            assert cut_rejects(xo, below, cut_hi)
        for _k in range(4):
            above = np.nextafter(above, f32(np.inf), dtype=np.float32)
            assert cut_rejects(xo, above, cut_hi)
        # the bounds themselves: a candidate at exactly xo +- reach is left out by
        # the upper cut (at or past the edge) and is rejected as well
        assert cut_rejects(xo, hi_x, cut_hi)


def test_the_reach_keeps_every_pair_inside_the_cut_off():
    # the cut never drops a pair the FP32 test could accept: any q with
    # fl((xo - q)^2) < cut_hi lies strictly within [lo_x, hi_x]
    rng = np.random.default_rng(8)
    for _ in range(2000):
        h = 10.0 ** rng.uniform(-4, 1)
        w = 2.0 * h * rng.uniform(1.0, 4.0 / 3.0)
        X = w * rng.integers(3, 129)
        cut_hi = f32((2.0 * h) ** 2 * (1.0 + 1e-5))
        reach = f32(f32(np.sqrt(cut_hi)) * f32(1.0 + 2.0 ** -12))
        xo = f32(rng.uniform(w, X - w))
        lo_x, hi_x = f32(xo - reach), f32(xo + reach)
        q = f32(xo - f32(rng.uniform(-1.0, 1.0)) * f32(np.sqrt(cut_hi)))
        if not cut_rejects(xo, q, cut_hi):
            assert lo_x < q < hi_x
