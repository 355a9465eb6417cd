"""The seeded input generators: sizes, structure and distributions of the
synthetic systems (the recipe the benchmark and the parity tests share),
checked against closed forms and textbook properties -- no GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2608_07327_amd import workloads as W


def _dense(A):
    return A.to_scipy().toarray()


def test_poisson2d_is_the_five_point_laplacian():
    m = 16
    A = W.poisson2d(m)
    assert A.n == m * m
    # 5 entries per row minus one per boundary side: 5 m^2 - 4 m
    assert A.nnz == 5 * m * m - 4 * m
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m, m))
    I = sp.identity(m)
    ref = (sp.kron(I, T) + sp.kron(T, I)).toarray()   # x fastest, as the generator orders
    assert np.array_equal(_dense(A), ref)
    # the benchmark's 64 x 64 case
    assert W.poisson2d(64).nnz == 20224


def test_diffusion3d_structure_and_coefficients():
    m = 9
    A = W.diffusion3d(m)
    n = m ** 3
    assert A.n == n
    # 7 entries per row, minus one per boundary face: 7 m^3 - 6 m^2
    assert A.nnz == 7 * n - 6 * m * m
    assert 7 * 128 ** 3 - 6 * 128 ** 2 == 14581760      # the 128^3 benchmark system
    D = _dense(A)
    assert np.array_equal(D, D.T)                       # harmonic-mean faces are symmetric
    # columns ascend within every row (the generator's slot order)
    for r in range(A.n):
        c = A.colind[A.rowptr[r]:A.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0.0)
    # row sums: zero in the interior, 2 kappa_c per Dirichlet face elsewhere
    rs = D.sum(axis=1)
    idx = np.arange(n)
    x, y, z = idx % m, (idx // m) % m, idx // (m * m)
    interior = (x > 0) & (x < m - 1) & (y > 0) & (y < m - 1) & (z > 0) & (z < m - 1)
    assert np.allclose(rs[interior], 0.0, atol=1e-12 * np.abs(np.diag(D)).max())
    assert np.all(rs[~interior] > 0.0)
    assert np.linalg.eigvalsh(D).min() > 0.0
    # the same tag gives the same bytes; sigma = 1 log-normal cell coefficients
    B = W.diffusion3d(m)
    assert np.array_equal(A.vals, B.vals) and np.array_equal(A.colind, B.colind)
    g = W.rng_for(W.CFG_DIFFUSION3D).standard_normal(n)
    kap = np.exp(g)
    # a corner cell: three Dirichlet faces (2 kappa) and three harmonic means
    c0 = 0
    nb = [1, m, m * m]
    want = 3 * 2 * kap[c0] + sum(2.0 / (1 / kap[c0] + 1 / kap[j]) for j in nb)
    assert np.isclose(D[c0, c0], want, rtol=1e-14)


def test_graph_laplacian_edges_degree_and_shift():
    n, deg, shift = 500, 8, 1e-2
    A = W.graph_laplacian(n, deg, shift, W.rng_for((70, 1)))
    D = _dense(A)
    assert A.nnz == n + n * deg                      # 4n distinct edges, both directions
    assert np.array_equal(D, D.T)
    assert np.allclose(D.sum(axis=1), shift)         # Laplacian rows sum to zero
    off = D - np.diag(np.diag(D))
    assert set(np.unique(off)) <= {-1.0, 0.0}        # unit weights, no self loops
    assert np.all(np.diag(off) == 0.0)
    assert np.isclose(np.linalg.eigvalsh(D).min(), shift, rtol=1e-6)


def test_graph_laplacian_batch_recipe():
    ys = W.graph_laplacian_batch(count=40, n_lo=100, n_hi=2000, tag=(71, 2))
    ns = np.array([y.A.n for y in ys])
    assert len(ys) == 40 and ns.min() >= 100 and ns.max() <= 2000
    assert {y.s for y in ys} <= {1, 4, 8}
    for y in ys[:5]:
        assert y.b.shape == (y.A.n,)


def test_dense_spd_is_bitwise_symmetric_with_the_shift_as_floor():
    n = 64
    A = W.dense_spd(n, tag=(72, 1), shift=1e-3)
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= 1e-3 * (1 - 1e-9)
    g = W.rng_for((72, 1)).standard_normal((n, n))
    ref = g @ g.T / n + 1e-3 * np.eye(n)
    # G is N(0,1) rounded to the 2^-8 grid: within 2^-9 of the draw per entry
    assert np.allclose(A, ref, rtol=0, atol=0.05)


@pytest.mark.parametrize("n", [64, 600, 1024])
def test_dense_spd_product_is_exact_and_blas_independent(n):
    """The entries of G are integers over 2^8, so G G^T computed in integer
    arithmetic is the exact product; numpy's BLAS and torch's matmul must
    both return exactly it (then any GPU BLAS does too)."""
    import torch
    g = W.dense_factor(n, (72, 2))
    k = np.rint(g * W.DENSE_GRID).astype(np.int64)
    assert np.array_equal(k / W.DENSE_GRID, g)
    exact = (k @ k.T).astype(np.float64) / W.DENSE_GRID ** 2
    A = W.dense_spd(n, tag=(72, 2), shift=1e-3)
    ref = exact / n
    ref[np.diag_indices(n)] += 1e-3
    assert np.array_equal(A, ref)
    At = W.dense_spd_torch(n, tag=(72, 2), shift=1e-3, device="cpu").numpy()
    assert np.array_equal(A, At)


def test_seeds_and_right_hand_sides():
    assert W.uniform_block_seed(3, 16) == 3016
    b1, b2 = W.rhs(1000, 5), W.rhs(1000, 5)
    assert np.array_equal(b1, b2)
    assert not np.array_equal(b1, W.rhs(1000, 6))
    big = W.rhs(200000, 9)
    assert abs(big.mean()) < 0.01 and abs(big.std() - 1.0) < 0.01


@pytest.mark.parametrize("cond", [10.0, 1e3])
def test_tiny_spd_has_the_requested_spectrum(cond):
    A = W.tiny_spd(12, cond, tag=(73, int(cond)))
    ev = np.linalg.eigvalsh(A)
    assert np.array_equal(A, A.T)
    assert np.allclose(ev, np.geomspace(1.0, cond, 12), rtol=1e-10)


def test_diffusion3d_inclusions_scale_the_cube_coefficients():
    m, k, size, contrast = 10, 3, 3, 1e4
    A0 = W.diffusion3d(m)
    A1 = W.diffusion3d(m, inclusions=k, contrast=contrast, size=size)
    # same sparsity, same coefficients outside the inclusions' neighbourhoods
    assert np.array_equal(A0.rowptr, A1.rowptr) and np.array_equal(A0.colind, A1.colind)
    D0, D1 = _dense(A0), _dense(A1)
    assert np.array_equal(D1, D1.T)
    assert np.linalg.eigvalsh(D1).min() > 0.0
    # rebuild the cells' coefficients the generator draws and check every
    # changed entry touches an inclusion cell
    n = m ** 3
    idx = np.arange(n)
    x, y, z = idx % m, (idx // m) % m, idx // (m * m)
    inside = np.zeros(n, dtype=bool)
    ri = W.rng_for((W.CFG_DIFFUSION3D, 77, m, k, size))
    for _ in range(k):
        c = ri.integers(1, m - size, 3)
        assert np.all(c >= 1) and np.all(c + size <= m - 1)
        inside |= ((x >= c[0]) & (x < c[0] + size) & (y >= c[1]) & (y < c[1] + size)
                   & (z >= c[2]) & (z < c[2] + size))
    assert size ** 3 <= inside.sum() <= k * size ** 3
    changed = np.argwhere(D0 != D1)
    assert len(changed) > 0
    # only rows of inclusion cells and of their neighbours change
    near = inside | ((D0 != 0).astype(int) @ inside.astype(int) > 0)
    assert np.all(near[changed[:, 0]]) and np.all(near[changed[:, 1]])
    # an interior inclusion cell's diagonal grows by about the contrast
    cell = np.flatnonzero(inside & (x > 0) & (x < m - 1) & (y > 0) & (y < m - 1)
                          & (z > 0) & (z < m - 1))
    assert D1[cell, cell].max() > 10.0 * D0[cell, cell].max()
