"""Pins of the four-colour Gauss-Seidel smoother of the oracle (cycle.colour_masks, smooth):
the colouring of a 5 x 5 grid against a hand-written fixture, and the defining property of one
colour step: point Gauss-Seidel solves each point's own equation, and points of one colour are
not coupled, so right after colour c's step the residual vanishes at every point of colour c
(for any colour order, on any stencil)."""
import os

import numpy as np
import pytest

import problems as pb
from oracle import boxmg, cycle, fem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "colour_masks_5x5.txt")


def test_colour_masks_match_hand_worked_5x5():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 5
    expected = np.full((5, 5), -1)
    for r, toks in enumerate(rows):
        j = 4 - r                                   # printed top row first
        for i, tok in enumerate(toks):
            expected[j, i] = -1 if tok == "." else int(tok)
    masks = cycle.colour_masks(5, 5)
    got = np.full(25, -1)
    for c, m in enumerate(masks):
        assert np.all(got[m] == -1), "a vertex in two colours"
        got[m] = c
    assert np.array_equal(got.reshape(5, 5), expected)


def test_same_colour_points_are_never_coupled():
    S = fem.assemble_stencil(*(lambda p: (p.jac, p.K))(pb.star(17, seed=3)), 17, 17)
    A = fem.stencil_to_matrix(S).tocoo()
    colour = np.full(17 * 17, -1)
    for c, m in enumerate(cycle.colour_masks(17, 17)):
        colour[m] = c
    off = (A.row != A.col) & (A.data != 0)
    assert np.all(colour[A.row[off]] != colour[A.col[off]])


@pytest.mark.parametrize("order", [(0, 1, 2, 3), (3, 2, 1, 0), (2, 0, 3, 1)])
@pytest.mark.parametrize("make", [lambda: pb.star(33, seed=2), lambda: pb.quarter_annulus(33),
                                  lambda: pb.discontinuous("checker", 33)])
def test_residual_vanishes_on_the_colour_just_smoothed(make, order):
    p = make()
    S = fem.assemble_stencil(p.jac, p.K, p.nx, p.ny)
    orc = cycle.Oracle(boxmg.build_hierarchy(S))
    A = orc.levels[0].A
    masks = orc.levels[0].masks
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, p.nx * p.ny)
    b = p.b.ravel().copy()
    for c in order:
        orc.smooth(0, u, b, (c,))
        r = b - A @ u
        scale = np.abs(b) + abs(A) @ np.abs(u)
        assert np.all(np.abs(r[masks[c]]) <= 1e-14 * scale[masks[c]]), c
        # the other colours are not solved (this is what the colour sweep leaves to the next one)
        others = masks[(c + 1) % 4]
        assert np.max(np.abs(r[others])) > 1e-8
