"""The biharmonic input operator (Section 7 problem F) against what the stencil fixes.

With unit spacing the 13-point stencil is exact on polynomials of degree <= 5:
rows whose whole stencil lies at least two nodes inside the grid must give
Delta^2 p exactly (0 for cubics, 24 for x^4, 8 for x^2 y^2).  Rows next to a
side see the mirrored node (Neumann) and the zero boundary node (Dirichlet):
checked on a hand-computed row.  The operator is symmetric positive definite.
"""

import numpy as np

from workloads.biharmonic import biharmonic13, biharmonic_problem


def _grid(m):
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    return i.ravel().astype(float), j.ravel().astype(float)


def test_stencil_exact_on_polynomials():
    m = 12
    A = biharmonic13(m).to_scipy()
    i, j = _grid(m)
    deep = (i >= 2) & (i <= m - 3) & (j >= 2) & (j <= m - 3)
    for u, lap2 in [(i ** 3 + 2 * i * j ** 2 - j, 0.0), (i ** 4, 24.0), (i ** 2 * j ** 2, 8.0),
                    (j ** 4 + i ** 4, 48.0), (i ** 5, None)]:
        r = A @ u
        if lap2 is None:
            assert np.allclose(r[deep], 120.0 * i[deep])   # Delta^2 x^5 = 120 x
        else:
            assert np.array_equal(r[deep], np.full(int(deep.sum()), lap2))


def test_rows_next_to_the_sides():
    m = 7
    A = biharmonic13(m).to_scipy().toarray()
    # corner node (0, 0): mirrored nodes on two sides, neighbours at -1 are boundary zeros
    r = A[0]
    assert r[0] == 22.0 and r[1] == -8.0 and r[m] == -8.0 and r[m + 1] == 2.0 and r[2] == 1.0 and r[2 * m] == 1.0
    assert np.count_nonzero(r) == 6
    # node (1, 3): one node from the side x = 0; its x - 2 neighbour is the boundary (zero)
    g = 1 + 3 * m
    r = A[g]
    assert r[g] == 20.0 and r[g - 1] == -8.0 and r[g + 1] == -8.0 and r[g + 2] == 1.0
    assert np.count_nonzero(r) == 12
    # node (0, 3): on the side x = 0, mirrored node adds one to the diagonal
    g = 3 * m
    assert A[g, g] == 21.0 and np.count_nonzero(A[g]) == 9


def test_spd_and_problem():
    A = biharmonic13(9).to_scipy().toarray()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    P = biharmonic_problem(24, 3, 1, 2)
    assert P.F.shape == (24 * 24, 6) and P.n_parts == 9 and P.rtol == 1e-6
