"""Pins of the oracle's Newell tensor against closed forms and quadratures
that share nothing with it (no GPU).  Cell-averaged demag tensor of Newell,
Williams & Dunlop, used for K = -N in eq. (7)/(12) of the paper."""
import itertools
import math

import numpy as np
import pytest

import oracle
from closed_forms import aharoni_diag, cellpair_gl, dipole_tensor


BOXES = [(1.0, 1.0, 1.0), (1.0, 1.3, 0.7), (4e-9, 4e-9, 2e-9), (3.90625e-9, 3.90625e-9, 3e-9),
         (2.0, 0.5, 0.25)]


@pytest.mark.parametrize("mode", ["exact", "q128"])
def test_cube_self_term_is_one_third(mode):
    for d in (1.0, 2e-9, 4e-9):
        N = oracle.newell(0, 0, 0, d, d, d, mode=mode)
        assert np.allclose(N[:3], 1.0 / 3.0, rtol=0, atol=1e-15)
        assert np.all(np.abs(N[3:]) <= 1e-15)


@pytest.mark.parametrize("box", BOXES)
def test_self_term_matches_aharoni_prism(box):
    """N(0) is the demag tensor of one cell: Aharoni's closed form."""
    N = oracle.newell(0, 0, 0, *box, mode="exact")
    D = aharoni_diag(*box)
    assert np.allclose(N[:3], D, rtol=1e-12, atol=0)
    assert abs(N[:3].sum() - 1.0) < 1e-13
    assert np.all(np.abs(N[3:]) <= 1e-14)


OFFSETS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 1, 1), (2, -1, 0), (3, 2, -1),
           (-5, 4, 2), (7, 0, -7), (12, -3, 5), (-20, 9, 14)]


@pytest.mark.parametrize("box", BOXES[:3])
@pytest.mark.parametrize("off", OFFSETS)
def test_trace_vanishes_off_origin(box, off):
    """Disjoint cells: the dipole kernel is traceless (Laplace), so is N."""
    R = [o * d for o, d in zip(off, box)]
    N = oracle.newell(*R, *box)
    assert abs(N[:3].sum()) <= 1e-9 * np.abs(N).max()


@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.0, 1.3, 0.7), (4e-9, 4e-9, 2e-9)])
def test_parity(box):
    """xx,yy,zz even in every axis; xy odd in X,Y; xz odd in X,Z; yz odd in Y,Z."""
    odd = {3: (0, 1), 4: (0, 2), 5: (1, 2)}
    for off in [(2, 1, 3), (1, 2, 0), (5, 3, 1), (9, 4, 2)]:
        R = np.array(off, dtype=float) * box
        N0 = oracle.newell(*R, *box)
        for flips in itertools.product((1, -1), repeat=3):
            Nf = oracle.newell(*(R * flips), *box)
            for c in range(6):
                s = 1.0
                if c in odd:
                    for a in odd[c]:
                        s *= flips[a]
                # equal up to the FP64 cancellation of the 27-term sum
                assert Nf[c] == pytest.approx(s * N0[c], rel=0, abs=1e-9 * np.abs(N0).max())


@pytest.mark.parametrize("off", [(2, 1, 0), (2, 0, 1), (0, 2, 1), (3, -2, 1), (2, 2, 2), (-2, 3, -1)])
@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.0, 1.3, 0.7)])
def test_nonadjacent_pair_matches_6d_quadrature(off, box):
    """Every component, off-diagonals included, equals a plain 6-D
    Gauss-Legendre average of the point-dipole kernel over the two cells."""
    R = [o * d for o, d in zip(off, box)]
    N = oracle.newell(*R, *box, mode="exact")
    G = cellpair_gl(R, box, n=12)
    assert np.allclose(N, G, rtol=0, atol=1e-11 * np.abs(G).max())


def test_far_field_tends_to_point_dipole():
    box = (1.0, 1.3, 0.7)
    V = box[0] * box[1] * box[2]
    u = np.array([0.6, -0.48, 0.64])
    prev = None
    for k in (8, 16, 32, 64, 128):
        R = k * u
        N = oracle.newell(*R, *box)
        D = dipole_tensor(R, V)
        err = np.abs(N - D).max() / np.abs(D).max()
        if prev is not None:
            assert err < prev / 3.0  # leading correction ~ (d/R)^2
        prev = err
    assert prev < 1e-4


@pytest.mark.parametrize("k", [8, 9, 12, 16])
def test_quadrature_matches_binary128_at_switch(k):
    for box in [(1.0, 1.0, 1.0), (4e-9, 4e-9, 2e-9)]:
        R = np.array([k, 0.37 * k, -0.21 * k]) * max(box)
        q = oracle.newell(*R, *box, mode="q128")
        f = oracle.newell(*R, *box, mode="far", p=4)
        assert np.abs(f - q).max() <= 1e-9 * np.abs(q).max()


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_exact_fp64_matches_binary128_near(k):
    for box in [(1.0, 1.0, 1.0), (1.0, 1.3, 0.7)]:
        R = np.array([k, 0.37 * k, 0.21 * k]) * max(box)
        q = oracle.newell(*R, *box, mode="q128")
        e = oracle.newell(*R, *box)
        assert np.abs(e - q).max() <= 1e-9 * np.abs(q).max()


@pytest.mark.parametrize("grid,box", [((3, 2, 2), (1.0, 1.3, 0.7)), ((4, 4, 4), (1.0, 1.0, 1.0)),
                                      ((5, 3, 1), (4e-9, 4e-9, 2e-9)), ((6, 2, 3), (2.0, 0.5, 0.25))])
def test_body_sum_is_prism_demag_factor(grid, box):
    """sum_{i,j} N(r_i - r_j) / n equals the demag tensor of the whole prism
    (Aharoni), off-diagonals zero: a uniformly magnetised prism."""
    nx, ny, nz = grid
    acc = np.zeros(6)
    cells = list(itertools.product(range(nx), range(ny), range(nz)))
    for a in cells:
        for b in cells:
            R = [(a[q] - b[q]) * box[q] for q in range(3)]
            acc += oracle.newell(*R, *box)
    acc /= len(cells)
    D = aharoni_diag(nx * box[0], ny * box[1], nz * box[2])
    assert np.allclose(acc[:3], D, rtol=1e-11)
    assert np.all(np.abs(acc[3:]) < 1e-13)


def test_block_additivity_off_diagonal():
    """Mutual tensor of two 2x2x2-cell blocks = Newell tensor of the blocks."""
    d = (1.0, 1.3, 0.7)
    big = tuple(2 * x for x in d)
    for boff in [(1, 1, 0), (1, 0, 1), (2, 1, -1)]:
        acc = np.zeros(6)
        for a in itertools.product(range(2), repeat=3):
            for b in itertools.product(range(2), repeat=3):
                R = [(2 * boff[q] + a[q] - b[q]) * d[q] for q in range(3)]
                acc += oracle.newell(*R, *d, mode="q128")
        acc /= 8.0
        Rb = [boff[q] * big[q] for q in range(3)]
        ref = oracle.newell(*Rb, *big, mode="q128")
        assert np.allclose(acc, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_octant_table_layout():
    nx, ny, nz = 5, 4, 3
    d = (1.0, 1.3, 0.7)
    T = oracle.tensor_octant(nx, ny, nz, *d)
    for (i, j, k) in [(0, 0, 0), (4, 3, 2), (2, 1, 0), (1, 3, 2)]:
        assert np.array_equal(T[:, k, j, i], oracle.newell(i * d[0], j * d[1], k * d[2], *d))
