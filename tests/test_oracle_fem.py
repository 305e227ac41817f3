"""Pins of the oracle's P1 assembly: the integer five-point stencil, exact
reproduction of linear functions on a distorted mesh, and second-order
convergence to a manufactured solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from paper_2310_14649_amd.inputs import jittered_mesh, structured_mesh


def test_unit_coefficient_gives_five_point_stencil():
    m = structured_mesh(6)
    K = fem.assemble(m.xy, m.tri, m.dof, m.n, np.ones((1, m.n_tri)))[0].toarray()
    a = 2 * 5 + 2                                  # interior node (3, 3)
    row = K[a]
    assert row[a] == pytest.approx(4.0, abs=1e-14)
    for b in (a - 1, a + 1, a - 5, a + 5):
        assert row[b] == pytest.approx(-1.0, abs=1e-14)
    # hypotenuse neighbours carry an exact zero
    assert row[a + 6] == 0.0 and row[a - 6] == 0.0
    assert np.count_nonzero(row) == 5


def test_element_areas_tile_the_square():
    for m in (structured_mesh(7), jittered_mesh(7, seed=4)):
        area, _ = fem.element_geometry(m.xy, m.tri)
        assert (area > 0).all()
        assert area.sum() == pytest.approx(1.0, abs=1e-14)


def test_linear_functions_in_kernel_on_jittered_mesh():
    """Rows of interior vertices of the full (boundary-inclusive) P1
    stiffness with a constant coefficient annihilate linear functions: checks
    the gradient formulas on non-right triangles."""
    m = jittered_mesh(9, seed=1)
    alldof = np.arange(m.n_vert, dtype=np.int32)
    c = np.full((1, m.n_tri), 2.5)
    K = fem.assemble(m.xy, m.tri, alldof, m.n_vert, c)[0]
    inner = m.dof >= 0
    for lin in (m.xy[:, 0], m.xy[:, 1], 2.0 * m.xy[:, 0] - 3.0 * m.xy[:, 1] + 1.0):
        assert np.abs((K @ lin)[inner]).max() < 1e-12
    # and a boundary row does not (the flux term): the check has teeth
    assert np.abs((K @ m.xy[:, 0])[~inner]).max() > 1e-3


def test_manufactured_solution_second_order():
    """-div(c grad u) = f with u = sin(pi x) sin(pi y), c = 1 + x y; the
    nodal error of P1 with lumped load and centroid coefficient is O(h^2)."""
    errs = []
    for nc in (8, 16, 32):
        m = structured_mesh(nc)
        cen = m.centroids()
        c = 1.0 + cen[:, 0] * cen[:, 1]
        x, y = m.xy[:, 0], m.xy[:, 1]
        pi = np.pi
        u = np.sin(pi * x) * np.sin(pi * y)
        ux = pi * np.cos(pi * x) * np.sin(pi * y)
        uy = pi * np.sin(pi * x) * np.cos(pi * y)
        f = (1 + x * y) * 2 * pi * pi * u - (y * ux + x * uy)
        K = fem.assemble(m.xy, m.tri, m.dof, m.n, c[None, :])[0]
        F = fem.load_vector_nodal(m.xy, m.tri, m.dof, m.n, f)
        uh = spla.spsolve(K.tocsc(), F)
        ue = np.empty(m.n)
        ue[m.dof[m.dof >= 0]] = u[m.dof >= 0]
        errs.append(np.abs(uh - ue).max())
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.3 < r < 4.8 for r in rates), (errs, rates)


def test_constant_load():
    m = structured_mesh(5)
    F = fem.load_vector(m.xy, m.tri, m.dof, m.n)
    # every interior node of the "/" mesh touches 6 triangles of area h^2/2
    assert np.allclose(F, 6 * (1.0 / 25) / 2 / 3)
