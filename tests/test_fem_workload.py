"""The finite-element workload of Section 6 (Poisson and Helmholtz on P1
triangles of the unit square) against the figures of Table 8.  CPU only.

Both generated matrices reproduce the table's sparsity, Frobenius norm and
condition number to the printed digits.  The Helmholtz condition number
depends on which diagonal splits each grid cell (the mass matrix does, the
stiffness matrix does not), so it pins the triangulation as well; the
Poisson figures pin the stiffness assembly and the boundary treatment.
The relative nodal L2 error of the exact discrete solution is compared
with the table's error of the iterate within a factor 2 (the paper's iterate
stops at RSE 1e-6 and its error norm is not stated)."""
import json
import os

import numpy as np
import pytest

import workloads.generators as g

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table8():
    with open(os.path.join(GOLDEN, "paper_fem_table8.json")) as f:
        return json.load(f)


CASES = {"poisson": (25, 0.0, 1), "helmholtz": (50, 25.0, 4)}


@pytest.fixture(scope="module", params=sorted(CASES))
def fem(request):
    npts, k, mode = CASES[request.param]
    A, b, u, xy = g.fem_p1_unit_square(npts, k, mode)
    return request.param, npts, A, b, u, xy


def test_matrix_matches_table8(fem):
    name, npts, A, b, u, xy = fem
    t = table8()[name]
    N = A.shape[0]
    assert N == npts * npts
    assert 2 * (npts - 1) ** 2 == t["elements"]
    assert round(100 * (1 - A.nnz / N ** 2), 2) == t["sparsity_percent"]
    # seven significant digits are printed
    fro = np.sqrt((A.data ** 2).sum())
    assert abs(fro - t["fro"]) <= 5e-7 * t["fro"]
    s = np.linalg.svd(A.toarray(), compute_uv=False)
    assert abs(s[0] / s[-1] - t["cond"]) <= 5e-7 * t["cond"]


def test_structure(fem):
    name, npts, A, b, u, xy = fem
    bnd = (xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) | (xy[:, 1] == 1)
    Ad = A.toarray()
    # symmetric; boundary rows and columns are unit vectors; b vanishes there
    assert np.array_equal(Ad, Ad.T)
    assert np.array_equal(Ad[np.ix_(bnd, bnd)], np.eye(bnd.sum()))
    assert not Ad[np.ix_(bnd, ~bnd)].any()
    assert not b[bnd].any()
    # the stiffness part is the 5-point stencil whatever the diagonals:
    # interior rows of the Poisson matrix sum to 0 away from the boundary
    if name == "poisson":
        inner = ~bnd
        far = inner & (xy[:, 0] > 0.05) & (xy[:, 0] < 0.95) & (xy[:, 1] > 0.05) & (xy[:, 1] < 0.95)
        assert np.allclose(Ad[far].sum(axis=1), 0.0, atol=1e-12)
        assert np.allclose(np.diag(Ad)[inner], 4.0)


def test_discrete_solution_error(fem):
    name, npts, A, b, u, xy = fem
    t = table8()[name]
    x = np.linalg.solve(A.toarray(), b)
    err = np.linalg.norm(x - u) / np.linalg.norm(u)
    assert t["rel_l2"] / 2 <= err <= 2 * t["rel_l2"]
