"""Particle pairs at the FP64 cut-off in oblique directions, for tests of the
neighbour predicate.  For each pair the squared distance summed in axis order
with one rounding per operation lies on one side of (2h)^2, while an evaluation
that fuses a square into the running sum (a fused multiply-add, which a
compiler may choose) lies on the other.  A predicate that contracts would thus
drop or add these pairs; the oracle's brute force and the GPU lists must both
follow the plain sum."""
from fractions import Fraction

import numpy as np

H_OVER_DP = 1.3


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def r2_plain(d):
    r2 = d[0] * d[0]
    for x in d[1:]:
        r2 = r2 + x * x
    return r2


def r2_fused(d):
    """The fused orders a compiler may pick: each later square fused into the
    sum, or the first square fused onto the second."""
    a = d[0] * d[0]
    for x in d[1:]:
        a = _fma(x, x, a)
    b = _fma(d[0], d[0], d[1] * d[1])
    for x in d[2:]:
        b = _fma(x, x, b)
    return a, b


def cut2_of(dp):
    h = H_OVER_DP * dp
    return (2.0 * h) * (2.0 * h)


def pairs(dim, dp, n_pairs, seed):
    """n_pairs pairs (a, b), each at a random oblique direction, b moved by
    single ulps along x until the plain and a fused sum fall on opposite sides
    of (2h)^2; centres on a coarse grid inside the unit box."""
    rng = np.random.default_rng(seed)
    cut2 = cut2_of(dp)
    r = np.sqrt(cut2)
    grid = np.linspace(0.25, 0.75, 4)  # pairs stay inside the box: no wrap
    centres = np.array(np.meshgrid(*([grid] * dim), indexing="ij")).reshape(dim, -1).T
    rng.shuffle(centres)
    out = []
    for c in centres:
        if len(out) == n_pairs:
            break
        for _ in range(50):
            u = rng.normal(size=dim)
            u /= np.linalg.norm(u)
            if np.min(np.abs(u)) < 0.2:
                continue
            a = c + rng.uniform(-0.01, 0.01, dim)
            b0 = a + r * u
            found = None
            for k in range(-48, 49):
                b = b0.copy()
                step = np.inf if k > 0 else -np.inf
                for _ in range(abs(k)):
                    b[0] = np.nextafter(b[0], step)
                d = a - b
                plain = r2_plain(d) < cut2
                if any((f < cut2) != plain for f in r2_fused(d)):
                    found = (a, b)
                    break
            if found is not None:
                out.append(found)
                break
    return out


def state(dim, n_side, with_lattice, seed):
    """Cut-off pairs alone, or set into a jittered lattice (lattice points
    within 0.4 dp of a pair particle removed), in the periodic unit box."""
    dp = 1.0 / n_side
    pp = pairs(dim, dp, 12, seed)
    extra = np.array([q for ab in pp for q in ab])
    if not with_lattice:
        return dp, extra, pp
    rng = np.random.default_rng(seed + 100)
    axes = [np.arange(n_side) * dp + 0.5 * dp] * dim
    lat = np.array(np.meshgrid(*axes, indexing="ij")).reshape(dim, -1).T
    lat = lat + rng.uniform(-0.3 * dp, 0.3 * dp, lat.shape)
    dist = np.min(np.linalg.norm(lat[:, None, :] - extra[None, :, :], axis=2), axis=1)
    lat = lat[dist > 0.4 * dp]
    return dp, np.vstack([lat % 1.0, extra]), pp
