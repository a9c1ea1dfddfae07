"""Pins of the Q1 elasticity generator (inputs of the vector-valued workload)."""

import numpy as np

from workloads.elasticity import elasticity_q1, graph_grow_partition, q1_reference_stiffness
from workloads import seed_rng


def rigid_modes(coords):
    x, y, z = coords
    n = x.size
    R = []
    for c in range(3):
        v = np.zeros(3 * n)
        v[c::3] = 1.0
        R.append(v)
    for i, j in [(0, 1), (0, 2), (1, 2)]:
        v = np.zeros(3 * n)
        v[i::3] = -coords[j]
        v[j::3] = coords[i]
        R.append(v)
    return np.array(R).T


def test_reference_stiffness_kernel_is_rigid_motions():
    h = 0.25
    K = q1_reference_stiffness(h, 0.3)
    nodes = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float).T * h
    R = rigid_modes(nodes)
    assert np.abs(K @ R).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.all(ev[:6] < 1e-12 * ev[-1]) and np.all(ev[6:] > 1e-3 * ev[-1])
    assert np.array_equal(K, K.T)


def test_uniform_stretch_energy():
    # u = (eps x, 0, 0) on one element: energy = 1/2 (lambda + 2 mu) eps^2 h^3 (E = 1)
    h, nu, eps = 0.5, 0.3, 1e-2
    K = q1_reference_stiffness(h, nu)
    u = np.zeros(24)
    for a in range(8):
        u[3 * a] = eps * ((a >> 0) & 1) * h
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    assert abs(0.5 * u @ K @ u - 0.5 * (lam + 2 * mu) * eps ** 2 * h ** 3) <= 1e-12


def test_assembled_operator():
    P = elasticity_q1(6, part_dofs=(100, 300), min_dofs=100)
    A = P.A.to_scipy()
    nel = 6
    assert P.n == 3 * nel * (nel + 1) ** 2
    assert (A - A.T).nnz == 0 or abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev[0] > 0
    # rigid translations are annihilated on rows whose node does not touch the clamped face
    h = 1.0 / nel
    nx = nel + 1
    nodes = np.arange(nx ** 3)
    free = nodes % nx > 0
    fx = (nodes % nx)[free]
    coords = [fx * h, ((nodes // nx) % nx)[free] * h, (nodes // nx ** 2)[free] * h]
    R = rigid_modes(coords)
    far = np.repeat(fx >= 2, 3)
    assert np.abs((A @ R)[far]).max() <= 1e-10 * abs(A).max()
    # generating vectors: component c carries {1, x, y, z} e_c
    F = P.F
    assert F.shape == (P.n, 12)
    for c in range(3):
        other = [d for d in range(3) if d != c]
        for d in other:
            assert not np.any(F[d::3, 4 * c:4 * c + 4])
        assert np.allclose(F[c::3, 4 * c], 1.0)
        assert np.allclose(F[c::3, 4 * c + 1], coords[0])


def test_graph_grow_partition_sizes_and_connectivity():
    nx = 9
    free = np.ones(nx ** 3, dtype=bool)
    part = graph_grow_partition((nx, nx, nx), free, seed_rng(7, 5), 150, 400, 150)
    sizes = np.bincount(part) * 3
    assert part.min() == 0 and sizes.min() >= 150
    # renumbered by lowest node
    firsts = [np.flatnonzero(part == p)[0] for p in range(part.max() + 1)]
    assert firsts == sorted(firsts)
    # each subdomain is connected in the 26-neighbour graph
    coords = np.stack([np.arange(nx ** 3) % nx, (np.arange(nx ** 3) // nx) % nx, np.arange(nx ** 3) // nx ** 2], 1)
    for p in range(part.max() + 1):
        nodes = set(np.flatnonzero(part == p).tolist())
        start = next(iter(nodes))
        seen, stack = {start}, [start]
        while stack:
            v = stack.pop()
            cv = coords[v]
            for w in nodes:
                if w not in seen and np.abs(coords[w] - cv).max() <= 1:
                    seen.add(w)
                    stack.append(w)
        assert seen == nodes
