"""Pins of the oracle's string-averaging projections (Sec. II-D), on the CPU.

Each pin is a case where SAP reduces to something with an independent definition:
  * one string per row with weights w_t: one iteration is the weighted simultaneous
    projection x + lambda sum_t w_t r_t / ||a_t||^2 a_t (Cimmino), written here with
    scipy's sparse products;
  * lambda = 1 on a single row: the iterate lands on the row's hyperplane, also when the
    row stores a column twice;
  * a system whose rows store some columns as several entries gives the iterates of the
    same matrix with those entries summed (scipy's sum_duplicates): SAP acts on the
    matrix A, not on its storage;
  * one string, lambda = 1, a consistent square system: Kaczmarz converges to its
    solution;
  * a consistent system started at its solution stays there, for any strings, weights
    and relaxation;
  * rows of zeros change nothing; strings without rows return x_k;
  * one string: the result depends on the row order (a sequential method), many
    one-row strings: it does not.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O


def _random_csr(m, n, nnz_per_row, seed, allow_dup=False):
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(m):
        k = int(rng.integers(1, nnz_per_row + 1))
        c = rng.choice(n, size=k, replace=allow_dup)
        rows += [i] * k
        cols += list(c)
        vals += list(rng.uniform(0.1, 2.0, size=k))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


def _sap(A, b, x0, **kw):
    return O.sap(A.indptr, A.indices, A.data, b, A.shape[1], x0, **kw)


@pytest.mark.parametrize("relax", [0.1, 1.0, 1.7])
def test_one_row_strings_are_cimmino(relax):
    A = _random_csr(40, 25, 6, 1)
    rng = np.random.default_rng(2)
    b = rng.uniform(0, 10, 40)
    x0 = rng.uniform(0, 1, 25)
    w = rng.uniform(0.5, 1.5, 40)
    w /= w.sum()
    got = _sap(A, b, x0, n_strings=40, relax=relax, weights=w)
    nrm = np.asarray(A.multiply(A).sum(axis=1)).ravel()
    r = b - A @ x0
    want = x0 + relax * (A.T @ (w * r / nrm))
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)
    # uniform weights: the default
    got_u = _sap(A, b, x0, n_strings=40, relax=relax)
    want_u = x0 + relax * (A.T @ (r / nrm)) / 40
    assert np.allclose(got_u, want_u, rtol=1e-12, atol=1e-12)


def test_unit_relaxation_projects_onto_the_row():
    A = _random_csr(1, 30, 12, 3)
    b = np.array([7.5])
    x0 = np.random.default_rng(4).uniform(0, 1, 30)
    x1 = _sap(A, b, x0, n_strings=1, relax=1.0)
    assert (A @ x1)[0] == pytest.approx(7.5, rel=1e-14)
    # the step is along the row: x1 - x0 is a multiple of a
    d = x1 - x0
    a = A.toarray()[0]
    k = d.dot(a) / a.dot(a)
    assert np.allclose(d, k * a, atol=1e-14)


def _split_entries(A, seed):
    """The same matrix with the first and about a third of the other entries of every row
    stored as two entries of the same column (value v as v * f and v * (1 - f)), the
    second one later in the row."""
    rng = np.random.default_rng(seed)
    rp, cols, vals = [0], [], []
    for i in range(A.shape[0]):
        c = list(A.indices[A.indptr[i]:A.indptr[i + 1]])
        v = list(A.data[A.indptr[i]:A.indptr[i + 1]])
        extra_c, extra_v = [], []
        for k in range(len(c)):
            if k == 0 or rng.uniform() < 0.35:
                f = rng.uniform(0.2, 0.8)
                extra_c.append(c[k])
                extra_v.append(v[k] * (1 - f))
                v[k] *= f
        cols += c + extra_c
        vals += v + extra_v
        rp.append(len(cols))
    return np.array(rp, np.int64), np.array(cols, np.int32), np.array(vals, np.float64)


def test_unit_relaxation_projects_onto_a_row_with_repeated_columns():
    A = _random_csr(1, 30, 12, 13)
    rp, cols, vals = _split_entries(A, 14)
    assert len(cols) > A.nnz
    b = np.array([7.5])
    x0 = np.random.default_rng(15).uniform(0, 1, 30)
    x1 = O.sap(rp, cols, vals, b, 30, x0, n_strings=1, relax=1.0)
    assert (A @ x1)[0] == pytest.approx(7.5, rel=1e-14)
    d = x1 - x0
    a = A.toarray()[0]
    assert np.allclose(d, d.dot(a) / a.dot(a) * a, atol=1e-14)


@pytest.mark.parametrize("M,relax", [(1, 1.0), (4, 0.3), (40, 1.5)])
def test_repeated_entries_act_as_their_sum(M, relax):
    A = _random_csr(40, 25, 8, 16)
    rp, cols, vals = _split_entries(A, 17)
    b = np.random.default_rng(18).uniform(0, 10, 40)
    x0 = np.random.default_rng(19).uniform(0, 1, 25)
    want = _sap(A, b, x0, n_strings=M, relax=relax, n_iter=3)
    got = O.sap(rp, cols, vals, b, 25, x0, n_strings=M, relax=relax, n_iter=3)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_kaczmarz_converges_on_consistent_square_system():
    rng = np.random.default_rng(5)
    n = 12
    M_ = rng.uniform(-1, 1, (n, n)) + 4 * np.eye(n)
    A = sp.csr_matrix(M_)
    xs = rng.uniform(0, 2, n)
    b = A @ xs
    x = _sap(A, b, np.zeros(n), n_strings=1, relax=1.0, n_iter=300)
    assert np.allclose(x, xs, atol=1e-10)


@pytest.mark.parametrize("M,relax", [(1, 0.1), (3, 0.5), (7, 1.9), (50, 1.0)])
def test_solution_is_a_fixed_point(M, relax):
    A = _random_csr(50, 30, 8, 6)
    xs = np.random.default_rng(7).uniform(0, 2, 30)
    b = A @ xs
    w = np.random.default_rng(8).uniform(0.2, 1.0, M)
    w /= w.sum()
    x = _sap(A, b, xs, n_strings=M, relax=relax, weights=w, n_iter=3)
    assert np.allclose(x, xs, rtol=1e-13, atol=1e-13)


def test_zero_rows_and_empty_strings():
    A = _random_csr(6, 10, 4, 9).tolil()
    A[2, :] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    b = np.arange(6, dtype=float)
    x0 = np.linspace(0, 1, 10)
    # dropping the zero row from its string changes nothing
    keep = np.array([0, 1, 3, 4, 5])
    a1 = _sap(A, b, x0, n_strings=1, relax=0.7)
    a2 = _sap(A[keep], b[keep], x0, n_strings=1, relax=0.7)
    assert np.array_equal(a1, a2)
    # 6 rows in 10 strings: 4 strings are empty and return x0
    w = np.full(10, 0.1)
    got = _sap(A, b, x0, n_strings=10, relax=0.7, weights=w)
    s = [t * 6 // 10 for t in range(11)]
    want = np.zeros(10)
    for t in range(10):
        rows = list(range(s[t], s[t + 1]))
        y = x0.copy() if not rows else _sap(A[rows], b[rows], x0, n_strings=1, relax=0.7)
        want += 0.1 * y
    assert np.allclose(got, want, rtol=1e-14, atol=1e-14)


def test_row_order():
    A = _random_csr(30, 20, 6, 10)
    b = np.random.default_rng(11).uniform(0, 5, 30)
    x0 = np.zeros(20)
    perm = np.random.default_rng(12).permutation(30)
    seq = _sap(A, b, x0, n_strings=1, relax=1.0)
    seq_p = _sap(A, b, x0, n_strings=1, relax=1.0, order=perm)
    seq_ref = _sap(A[perm], b[perm], x0, n_strings=1, relax=1.0)
    assert np.allclose(seq_p, seq_ref, rtol=1e-14, atol=1e-14)
    assert not np.allclose(seq, seq_p)
    sim = _sap(A, b, x0, n_strings=30, relax=1.0)
    sim_p = _sap(A, b, x0, n_strings=30, relax=1.0, order=perm)
    assert np.allclose(sim, sim_p, rtol=1e-12, atol=1e-12)


def test_reconstruction_approaches_phantom():
    """A small consistent pCT system: the SAP iterates approach the true x."""
    from paper_2108_12369_amd import workloads as W
    ph = W.phantom(2, (40, 32), (5.0, 5.0), W.neo1_regions())
    bm = W.beam(31, 36, 5.0, 36 * 120, (-125.0, 125.0))
    o = O.run(W.workload("sap-pin", ph, bm))
    x_true = o["x"].astype(np.float64)
    b = o["b"]
    errs = []
    x = np.zeros_like(x_true)
    for _ in range(4):
        x = O.sap(o["row_ptr"], o["cols"], o["vals"], b, len(x_true), x, n_strings=20, relax=0.5,
                  n_iter=5)
        errs.append(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 0.15
