"""Comparison of a mixed-precision GPU simulation with the FP64 oracle, shared
by the GPU tests: per-particle bars, cell-flip and accept-flip accounting (see
test_gpu_mixed.py for the bars and the reasons behind them)."""
import numpy as np

TOL = 1e-5
NEAR_TIE = 2.0**-22


def by_id(ids, arr):
    out = np.empty_like(arr)
    out[..., ids] = arr
    return out


class Tracker:
    """Free-running comparison of a mixed GPU simulation with the oracle,
    called after every step: particles whose cell differs, the other particles
    of the cells such a particle is in (either side), and from then on every
    particle that shares a cell with an excluded one, leave the comparison."""

    def __init__(self, prob, disc):
        self.prob, self.disc = prob, disc
        self.h = prob["L"][0] / disc["nc"][0]
        self.excluded = np.zeros(disc["np"], dtype=bool)
        self.flips = 0

    def check(self, P, g, o, tag=""):
        disc, prob, h = self.disc, self.prob, self.h
        ncell = int(np.prod(disc["nc"]))
        ig, io = g.get(P.STATE_ID), o.get(o.ID)
        cg = by_id(ig, np.repeat(np.arange(ncell), np.diff(g.get(P.STATE_CELL_START))))
        co = by_id(io, np.repeat(np.arange(ncell), np.diff(o.get(o.CELL_START))))
        xg, xo = by_id(ig, g.get(P.STATE_X)), by_id(io, o.get(o.X))
        vg, vo = by_id(ig, g.get(P.STATE_V)), by_id(io, o.get(o.V))
        flipped = cg != co
        if flipped.any():
            # a flipped particle sits at a face of its oracle cell
            s = xo[:, flipped] / h
            frac = s - np.floor(s)
            face = np.minimum(frac, 1.0 - frac).min(axis=0)
            assert np.all(face <= TOL), f"{tag}: cell flip away from a face ({face.max():.2e} h)"
            self.flips += int(flipped.sum())
        bad_cells = np.union1d(cg[flipped | self.excluded], co[flipped | self.excluded])
        self.excluded |= np.isin(cg, bad_cells) | np.isin(co, bad_cells)
        keep = ~self.excluded
        dx = np.abs(xg - xo)
        dx = np.minimum(dx, np.array(prob["L"])[:, None] - dx).max(axis=0)
        dv = np.abs(vg - vo).max(axis=0)
        assert self.flips <= 4, f"{tag}: {self.flips} cell flips"
        mx, mv = dx[keep].max() / h, dv[keep].max() / prob["vbar"]
        assert mx <= TOL and mv <= TOL, f"{tag}: max dx/h {mx:.2e}, dv/vbar {mv:.2e} " \
            f"({int((dx[keep] > TOL * h).sum() + (dv[keep] > TOL * prob['vbar']).sum())} outliers)"
        return mx, mv


def first_flips_are_near_ties(a, b, ties):
    """a, b: pair logs (n, 7) of the GPU and the oracle in the same (sorted)
    order; ties: the oracle's (U, ratio) per pair in that order.  The first
    differing accept decision of each (cell, call, outcome) must be a
    near-tie.  Returns the number of differing decisions."""
    diff = np.nonzero(a[:, 6] != b[:, 6])[0]
    seen = set()
    for i in diff:
        key = (int(b[i, 0]), int(b[i, 1]), int(b[i, 2]))
        if key in seen:
            continue
        seen.add(key)
        u, r = ties[i]
        assert abs(u - r) <= NEAR_TIE, f"accept flip at {key} is not a near-tie: U {u}, ratio {r}"
    return len(diff)


def sorted_pairs(log, ties=None):
    a = np.asarray(log, dtype=np.int64).reshape(-1, 7)
    order = np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))
    return (a[order], None if ties is None else ties[order])
