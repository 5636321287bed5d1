"""Pins for the FP64 oracle: the paper's worked examples (tests/golden/),
closed forms, special cases that reduce to library routines (numpy einsum /
matmul), identities fixed by the definitions, and brute force on tiny inputs.
None of these uses the HIP library."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield [c.strip() for c in line.split(";")]


def _ints(s):
    return tuple(int(v) for v in s.split(","))


def _rand_layout(p, g):
    return synth.random_layout(p, g)


def _einsum_ttt(A, B, q, phi, psi):
    """Eq. ttt / ttt_indices expressed as one numpy.einsum call."""
    letters = "abcdefghijklmnopqrstuvwxyz"
    pa, pb = A.ndim, B.ndim
    r, s = pa - q, pb - q
    la = [None] * pa
    lb = [None] * pb
    it = iter(letters)
    out = []
    for k in range(r):
        la[phi[k] - 1] = next(it)
        out.append(la[phi[k] - 1])
    for k in range(s):
        lb[psi[k] - 1] = next(it)
        out.append(lb[psi[k] - 1])
    for k in range(q):
        c = next(it)
        la[phi[r + k] - 1] = c
        lb[psi[s + k] - 1] = c
    spec = "%s,%s->%s" % ("".join(la), "".join(lb), "".join(out))
    return np.einsum(spec, np.asarray(A), np.asarray(B))


# ------------------------------------------------------------ paper examples

def test_strides_golden():
    for shape, layout, w in _rows("strides.txt"):
        assert oracle.strides(_ints(shape), _ints(layout)) == _ints(w)


def test_first_and_last_order_equations():
    # Sec. 3.1 Eq. stride.tuple.first.order and stride.tuple.last.order
    n = (3, 5, 2, 7)
    assert oracle.strides(n) == (1, 3, 15, 30)
    assert oracle.strides(n, oracle.last_order(4)) == (70, 14, 7, 1)


def test_fiber_golden():
    for shape, layout, fixed, mem in _rows("fiber.txt"):
        n, w = _ints(shape), oracle.strides(_ints(shape), _ints(layout))
        fixed = fixed.split(",")
        run = fixed.index("*")
        idx = [0 if v == "*" else int(v) for v in fixed]
        got = []
        for i in range(n[run]):
            idx[run] = i
            got.append(sum(a * b for a, b in zip(w, idx)))
        assert tuple(got) == _ints(mem)


def test_view_golden():
    kv = {}
    elems = []
    for row in _rows("view.txt"):
        if row[0] == "element":
            elems.append((_ints(row[1]), _ints(row[2])))
        else:
            kv[row[0]] = _ints(row[1])
    n, pi = kv["shape"], kv["layout"]
    f, t, l = kv["first"], kv["step"], kv["last"]
    nv = tuple((l[r] - f[r]) // t[r] + 1 for r in range(3))  # Eq. view_extent
    assert nv == kv["view_shape"]
    w = oracle.strides(n, pi)
    gamma = sum(w[r] * f[r] for r in range(3))  # Eq. view_gamma with o = 0
    assert (gamma,) == kv["gamma"]
    wv = tuple(w[r] * t[r] for r in range(3))
    assert wv == kv["view_strides"]
    # parent holds a code of its multi-index; copy the view through the oracle
    parent = oracle.empty(n, pi)
    for i in itertools.product(*[range(v) for v in n]):
        parent[i] = 100 * i[0] + 10 * i[1] + i[2]
    flat = np.lib.stride_tricks.as_strided(parent, shape=(parent.size,), strides=(8,))
    view = np.lib.stride_tricks.as_strided(flat[gamma:], shape=nv, strides=tuple(8 * s for s in wv))
    dense = oracle.scale(1.0, view)
    for iv, ip in elems:
        assert dense[iv] == 100 * ip[0] + 10 * ip[1] + ip[2]


def _matlab_tensor():
    kv, rows = {}, []
    for row in _rows("matlab_stream.txt"):
        if row[0] in ("shape", "layout"):
            kv[row[0]] = _ints(row[1])
        else:
            rows.append((int(row[0]), int(row[1]), [float(v) for v in row[2].split()]))
    n, pi = kv["shape"], kv["layout"]
    A = oracle.empty(n, pi)
    flat = np.lib.stride_tricks.as_strided(A, shape=(A.size,), strides=(8,))
    flat[:] = np.arange(A.size, dtype=np.float64)  # memory element j holds j
    return A, rows


def test_matlab_stream_golden():
    A, rows = _matlab_tensor()
    first = oracle.scale(1.0, A, pi=[1, 2, 3])  # relayout to first order through the oracle
    for i3, i1, vals in rows:
        assert [first[i1, i2, i3] for i2 in range(4)] == vals


def test_ttv_closed_forms_on_matlab_example():
    # A(i1,i2,i3) = 8 i1 + 2 i2 + i3, shape (3,4,2); b = ones
    A, _ = _matlab_tensor()
    c1 = oracle.ttv(A, np.ones(3), 1)
    c2 = oracle.ttv(A, np.ones(4), 2)
    c3 = oracle.ttv(A, np.ones(2), 3)
    for i2 in range(4):
        for i3 in range(2):
            assert c1[i2, i3] == 24 + 6 * i2 + 3 * i3
    for i1 in range(3):
        for i3 in range(2):
            assert c2[i1, i3] == 32 * i1 + 12 + 4 * i3
    for i1 in range(3):
        for i2 in range(4):
            assert c3[i1, i2] == 16 * i1 + 4 * i2 + 1


def test_inner_on_matlab_example():
    A, _ = _matlab_tensor()
    assert oracle.inner(A, A) == sum(j * j for j in range(24)) == 4324


def test_member_function_shapes():
    g = synth.rng(99, 0)
    for op, sa, sb, ma, mb, sc in _rows("member_shapes.txt"):
        A = synth.uniform(_ints(sa), g)
        B = synth.uniform(_ints(sb), g)
        if op == "ttv":
            C = oracle.ttv(A, B, int(ma))
        elif op == "ttm":
            C = oracle.ttm(A, B, int(ma))
        else:
            ca, cb = _ints(ma), _ints(mb)
            free_a = [k for k in range(1, A.ndim + 1) if k not in ca]
            free_b = [k for k in range(1, B.ndim + 1) if k not in cb]
            C = oracle.ttt(A, B, len(ca), free_a + list(ca), free_b + list(cb))
        assert C.shape == _ints(sc)


def test_superdiagonal_ttv_is_diag():
    # Sec. 3.2 Example superdiagonal: A(i,i,i) = 1; mode-1 TTV with b gives diag(b)
    n = 5
    for pi in ([1, 2, 3], [3, 2, 1], [2, 3, 1]):
        A = oracle.empty((n, n, n), pi)
        for i in range(n):
            A[i, i, i] = 1.0
        b = np.arange(1.0, n + 1)
        for m in (1, 2, 3):
            C = oracle.ttv(A, b, m)
            np.testing.assert_array_equal(np.asarray(C), np.diag(b))


# ------------------------------------------------------------ library routines

@pytest.mark.parametrize("seed", range(6))
def test_ttv_vs_einsum(seed):
    g = synth.rng(98, seed)
    p = 2 + seed % 4
    n = tuple(int(v) for v in g.integers(1, 6, p))
    X = synth.uniform(n, g)
    A = oracle.materialize(X, _rand_layout(p, g))
    for m in range(1, p + 1):
        b = synth.uniform((n[m - 1],), g)
        C = oracle.ttv(A, b, m, pi=_rand_layout(p - 1, g))
        ref = np.tensordot(X, b, axes=([m - 1], [0]))
        np.testing.assert_allclose(np.asarray(C), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_ttm_vs_unfolding_matmul(seed):
    # C_(m) = B . A_(m): the mode-m unfolding turns TTM into a matrix product
    g = synth.rng(97, seed)
    p = 2 + seed % 4
    n = tuple(int(v) for v in g.integers(1, 6, p))
    X = synth.uniform(n, g)
    A = oracle.materialize(X, _rand_layout(p, g))
    for m in range(1, p + 1):
        B = synth.uniform((int(g.integers(1, 5)), n[m - 1]), g)
        C = oracle.ttm(A, B, m, pi=_rand_layout(p, g))
        unf = np.moveaxis(X, m - 1, 0).reshape(n[m - 1], -1)
        ref = np.moveaxis((B @ unf).reshape((B.shape[0],) + tuple(np.delete(n, m - 1))), 0, m - 1)
        np.testing.assert_allclose(np.asarray(C), ref, rtol=1e-13, atol=1e-13)


def _random_ttt(g, pa, pb, q):
    na = [int(v) for v in g.integers(1, 5, pa)]
    phi = [int(v) + 1 for v in g.permutation(pa)]
    psi = [int(v) + 1 for v in g.permutation(pb)]
    r, s = pa - q, pb - q
    nb = [int(v) for v in g.integers(1, 5, pb)]
    for k in range(q):
        nb[psi[s + k] - 1] = na[phi[r + k] - 1]
    return tuple(na), tuple(nb), phi, psi


@pytest.mark.parametrize("seed", range(12))
def test_ttt_vs_einsum(seed):
    g = synth.rng(96, seed)
    pa = int(g.integers(1, 5))
    pb = int(g.integers(1, 5))
    q = int(g.integers(0, min(pa, pb) + 1))
    if pa - q + pb - q == 0 and q == 0:
        q = 1
    na, nb, phi, psi = _random_ttt(g, pa, pb, q)
    X, Y = synth.uniform(na, g), synth.uniform(nb, g)
    A = oracle.materialize(X, _rand_layout(pa, g))
    B = oracle.materialize(Y, _rand_layout(pb, g))
    pc = pa + pb - 2 * q
    C = oracle.ttt(A, B, q, phi, psi, pi=_rand_layout(pc, g) if pc else None)
    np.testing.assert_allclose(np.asarray(C), _einsum_ttt(X, Y, q, phi, psi), rtol=1e-13,
                               atol=1e-13)


def test_ttt_flattened_matmul():
    # A_(free x contracted) . B_(contracted x free) for the order-4/order-3 case (shrunk)
    X, Y = synth.ttt_case(shrink=8)
    A = oracle.materialize(X, [3, 1, 4, 2])
    B = oracle.materialize(Y)
    C = oracle.ttt(A, B, 2, (1, 2, 3, 4), (3, 1, 2))
    na = X.shape
    ref = (X.reshape(na[0] * na[1], na[2] * na[3], order="F")
           @ Y.reshape(na[2] * na[3], Y.shape[2], order="F"))
    np.testing.assert_allclose(np.asarray(C).reshape(na[0] * na[1], -1, order="F"), ref,
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_axpby_and_transpose(seed):
    g = synth.rng(95, seed)
    p = 1 + seed
    n = tuple(int(v) for v in g.integers(1, 5, p))
    X, Y = synth.uniform(n, g), synth.uniform(n, g)
    A = oracle.materialize(X, _rand_layout(p, g))
    B = oracle.materialize(Y, _rand_layout(p, g))
    C = oracle.axpby(0.75, A, -2.0, B, pi=_rand_layout(p, g))
    np.testing.assert_allclose(np.asarray(C), 0.75 * X - 2.0 * Y, rtol=1e-15, atol=1e-15)
    tau = _rand_layout(p, g)
    T = oracle.transpose(A, tau, pi=_rand_layout(p, g))
    np.testing.assert_array_equal(np.asarray(T), np.transpose(X, [t - 1 for t in tau]))


# ------------------------------------------------------------ identities

def _rand(g, n, pi=None):
    return oracle.materialize(synth.uniform(n, g), pi)


def test_ttm_identity_matrix_returns_A():
    g = synth.rng(94, 0)
    A = _rand(g, (3, 4, 5, 2), [2, 4, 1, 3])
    for m in range(1, 5):
        C = oracle.ttm(A, np.eye(A.shape[m - 1]), m)
        np.testing.assert_array_equal(np.asarray(C), np.asarray(A))


def test_ttm_modes_commute_and_compose():
    g = synth.rng(94, 1)
    A = _rand(g, (4, 3, 5), [3, 1, 2])
    U = synth.uniform((2, 3), g)
    V = synth.uniform((6, 5), g)
    W = synth.uniform((3, 2), g)
    c1 = oracle.ttm(oracle.ttm(A, U, 2), V, 3)
    c2 = oracle.ttm(oracle.ttm(A, V, 3), U, 2)
    np.testing.assert_allclose(np.asarray(c1), np.asarray(c2), rtol=1e-13, atol=1e-13)
    # (A x_2 U) x_2 W = A x_2 (W U)
    c3 = oracle.ttm(oracle.ttm(A, U, 2), W, 2)
    c4 = oracle.ttm(A, W @ U, 2)
    np.testing.assert_allclose(np.asarray(c3), np.asarray(c4), rtol=1e-13, atol=1e-13)


def test_ttm_adjoint():
    # <A x_q U, Y> = <A, Y x_q U^T>
    g = synth.rng(94, 2)
    A = _rand(g, (3, 4, 5))
    U = synth.uniform((6, 4), g)
    Y = _rand(g, (3, 6, 5), [3, 2, 1])
    lhs = oracle.inner(oracle.ttm(A, U, 2), Y)
    rhs = oracle.inner(A, oracle.ttm(Y, np.ascontiguousarray(U.T), 2))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_ttm_with_one_row_is_ttv_and_p2_is_matmul():
    g = synth.rng(94, 3)
    A = _rand(g, (3, 4, 5), [2, 1, 3])
    b = synth.uniform((4,), g)
    c_ttm = oracle.ttm(A, b.reshape(1, 4), 2)
    c_ttv = oracle.ttv(A, b, 2)
    np.testing.assert_array_equal(np.asarray(c_ttm)[:, 0, :], np.asarray(c_ttv))
    M = _rand(g, (3, 4))
    B = synth.uniform((5, 4), g)
    np.testing.assert_allclose(np.asarray(oracle.ttm(M, B, 2)), np.asarray(M) @ B.T, rtol=1e-14)
    # TTV with p = 2, m = 1 is a vector-matrix product
    v = synth.uniform((3,), g)
    np.testing.assert_allclose(np.asarray(oracle.ttv(M, v, 1)), v @ np.asarray(M), rtol=1e-14)


def test_ttt_reductions():
    # Sec. 5.2: TTT reduces to TTV, to TTM with m = p, to the inner and the outer product
    g = synth.rng(94, 4)
    A = _rand(g, (3, 4, 5), [3, 1, 2])
    b = synth.uniform((4,), g)
    c = oracle.ttt(A, b, 1, (1, 3, 2), (1,))
    np.testing.assert_array_equal(np.asarray(c), np.asarray(oracle.ttv(A, b, 2)))
    B = synth.uniform((6, 5), g)
    c = oracle.ttt(A, B, 1, (1, 2, 3), (1, 2))
    np.testing.assert_array_equal(np.asarray(c), np.asarray(oracle.ttm(A, B, 3)))
    A2 = _rand(g, (3, 4, 5), [2, 3, 1])
    ip = oracle.ttt(A, A2, 3, (1, 2, 3), (1, 2, 3))
    assert abs(float(np.asarray(ip)) - oracle.inner(A, A2)) < 1e-13
    u, v = synth.uniform((3,), g), synth.uniform((4,), g)
    np.testing.assert_array_equal(np.asarray(oracle.ttt(u, v, 0, (1,), (1,))), np.outer(u, v))


def test_ttt_joint_pair_permutation_invariant():
    g = synth.rng(94, 5)
    X, Y = synth.ttt_case(shrink=8)
    A, B = oracle.materialize(X), oracle.materialize(Y, [2, 3, 1])
    c1 = oracle.ttt(A, B, 2, (1, 2, 3, 4), (3, 1, 2))
    c2 = oracle.ttt(A, B, 2, (1, 2, 4, 3), (3, 2, 1))
    np.testing.assert_allclose(np.asarray(c1), np.asarray(c2), rtol=1e-13, atol=1e-12)


def test_inner_norm_identities():
    g = synth.rng(94, 6)
    X = synth.uniform((7, 6, 5), g)
    A = oracle.materialize(X, [3, 1, 2])
    B = _rand(g, (7, 6, 5), [2, 1, 3])
    nA, nB = oracle.norm(A), oracle.norm(B)
    assert abs(oracle.inner(A, A) - nA * nA) <= 1e-13 * nA * nA
    assert abs(oracle.inner(A, B)) <= nA * nB  # Cauchy-Schwarz
    assert oracle.inner(A, A) == math.fsum(float(v) * float(v) for v in X.reshape(-1, order="F"))


def test_inner_compensated_vs_fsum():
    g = synth.rng(94, 7)
    X = synth.uniform((64, 64, 16), g) * np.exp(g.uniform(-8, 8, (64, 64, 16)))
    Y = synth.uniform((64, 64, 16), g)
    A, B = oracle.materialize(X), oracle.materialize(Y, [3, 2, 1])
    exact = math.fsum((X * Y).reshape(-1))
    assert abs(oracle.inner(A, B) - exact) <= 4e-16 * np.abs(X * Y).sum()


def test_layout_invariance_bitwise():
    # the summation order only depends on multi-indices, so every layout of the
    # same logical tensor gives bitwise identical results
    g = synth.rng(94, 8)
    X = synth.uniform((5, 4, 6, 3), g)
    b = synth.uniform((6,), g)
    B = synth.uniform((7, 4), g)
    outs_v, outs_m = [], []
    for pi in ([1, 2, 3, 4], [4, 3, 2, 1], [3, 1, 4, 2]):
        A = oracle.materialize(X, pi)
        outs_v.append(np.asarray(oracle.ttv(A, b, 3)).copy())
        outs_m.append(np.asarray(oracle.ttm(A, B, 2)).copy())
    for o in outs_v[1:]:
        np.testing.assert_array_equal(o, outs_v[0])
    for o in outs_m[1:]:
        np.testing.assert_array_equal(o, outs_m[0])


def test_integer_inputs_exact():
    g = synth.rng(94, 9)
    X = synth.integers((6, 5, 7), g)
    A = oracle.materialize(X, [2, 3, 1])
    B = synth.integers((4, 5), g)
    C = oracle.ttm(A, B, 2)
    ref = np.einsum("ijk,lj->ilk", X.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(np.asarray(C), ref.astype(np.float64))


def test_brute_force_tiny_ttt():
    # dictionary-based brute force over Eq. ttt on a 2x3x2 / 3x2x2 pair
    g = synth.rng(94, 10)
    X, Y = synth.uniform((2, 3, 2), g), synth.uniform((3, 2, 2), g)
    phi, psi = (1, 2, 3), (3, 1, 2)   # free A mode 1, free B mode 3; pairs (2,1), (3,2)
    C = oracle.ttt(oracle.materialize(X, [3, 2, 1]), oracle.materialize(Y), 2, phi, psi)
    for i in range(2):
        for k in range(2):
            acc = 0.0
            for j1 in range(3):
                for j2 in range(2):
                    acc += X[i, j1, j2] * Y[j1, j2, k]
            assert abs(C[i, k] - acc) < 1e-14


# ------------------------------------------------------------ drivers

def test_hopm_rank_one_closed_form():
    # A = sigma a o b o c o d: one sweep returns lambda = sigma and the factors (up to sign)
    g = synth.rng(94, 11)
    fac = [synth.orthonormal_columns(n, 1, g)[:, 0] for n in (5, 4, 6, 3)]
    sigma = 7.5
    X = sigma * np.einsum("i,j,k,l->ijkl", *fac)
    A = oracle.materialize(X, [2, 4, 1, 3])
    us = [np.full(n, 1.0 / math.sqrt(n)) for n in X.shape]
    lam, u = oracle.hopm(A, us, 1)
    assert abs(lam[-1] - sigma) < 1e-12 * sigma
    for k in range(4):
        assert abs(abs(float(np.dot(u[k], fac[k]))) - 1.0) < 1e-12


def test_times_vectors_vs_einsum():
    g = synth.rng(94, 12)
    X = synth.uniform((3, 4, 5, 2), g)
    A = oracle.materialize(X, [4, 2, 3, 1])
    us = [synth.uniform((n,), g) for n in X.shape]
    for r in range(1, 5):
        v = oracle.times_vectors(A, us, r)
        spec = "ijkl," + ",".join(c for k, c in enumerate("ijkl") if k != r - 1) + "->" + "ijkl"[r - 1]
        ref = np.einsum(spec, X, *[us[k] for k in range(4) if k != r - 1])
        np.testing.assert_allclose(v, ref, rtol=1e-13, atol=1e-13)


def test_tucker_vs_einsum_and_norm_bound():
    g = synth.rng(94, 13)
    A, Us, F, sig = synth.tucker_case(n=16, rank=3, rows=4, sigma0=10.0, noise=0.01, g=g)
    At = oracle.materialize(A)
    core = oracle.tucker(At, Us)
    ref = np.einsum("ijkl,ai,bj,ck,dl->abcd", A, *Us)
    np.testing.assert_allclose(np.asarray(core), ref, rtol=1e-12, atol=1e-12)
    assert oracle.norm(core) <= oracle.norm(At) * (1 + 1e-12)


def test_errors():
    A = oracle.empty((3, 4))
    with pytest.raises(ValueError):
        oracle.ttv(A, np.ones(5), 2)
    with pytest.raises(ValueError):
        oracle.ttm(A, np.ones((2, 3)), 2)
    with pytest.raises(ValueError):
        oracle.strides((2, 3), (1, 1))
    with pytest.raises(ValueError):
        oracle.ttt(A, oracle.empty((5, 2)), 1, (1, 2), (1, 2))
