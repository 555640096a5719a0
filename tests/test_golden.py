"""Fixtures under tests/golden/: values fixed by the paper's formulas or by textbook closed forms,
each file citing the passage it follows (no stored value comes from the library)."""
import os

import numpy as np

import problems as pb
from oracle import fem, transfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


def test_quarter_annulus_map_inverts_the_papers_T():
    """X(T(x)) = x at points where the paper's T has a closed form."""
    mp = pb.QuarterAnnulus()
    for x, y, xi, eta in _rows("quarter_annulus_T.txt"):
        X, Y = mp(xi, eta)
        assert abs(X - x) < 1e-15 and abs(Y - y) < 1e-15, (x, y, xi, eta)


def test_constant_tensor_stencils():
    for J11, J12, J21, J22, a, b, c, *ref in _rows("q1_constant_tensor_stencil.txt"):
        mp = pb.Affine(np.array([[J11, J12], [J21, J22]]))
        M11, M12, M22 = fem.metric_tensor(*mp.jacobian(0.0, 0.0))
        assert np.allclose([M11, M12, M22], [a, b, c], atol=1e-15)
        jac = pb.sample_jacobian(mp, 9, 9)
        S = fem.assemble_stencil(jac, np.ones((8, 8)), 9, 9)
        for k in range(5):
            assert np.allclose(S[k][2:-2, 2:-2], ref[k], atol=1e-14), (J11, J12, J21, J22, k)


def test_p1_element_mass():
    for x0, y0, x1, y1, x2, y2, *m in _rows("p1_element_mass.txt"):
        xy = np.array([[x0, y0], [x1, y1], [x2, y2]])
        M = transfer.p1_mass(xy, np.array([[0, 1, 2]], dtype=np.int32), np.ones(3, dtype=bool)).toarray()
        ref = np.array([[m[0], m[1], m[2]], [m[1], m[3], m[4]], [m[2], m[4], m[5]]])
        assert np.allclose(M, ref, atol=1e-16)
