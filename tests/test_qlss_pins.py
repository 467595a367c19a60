"""QLSS building blocks (paper_2503_15118_amd/qlss.py) on the CPU oracle:
controlled state preparation from binary-tree angles read from QRAM, the
block encoding U_A = U_SWAP U_R^dagger U_L with
<i|<0|<0| U_A |j>|0>|0> = A_ij / ||A||_F, and the walk step R U_A; the oracle
against the dense checker on a small instance."""
import numpy as np
import pytest

import workloads as wl
from oracle.dense import DenseState
from oracle.oracle import OracleState
from paper_2503_15118_amd.qlss import block_encoding, circuit, dequantize, tree_angles, walk_step


def _matrix(seed, n, density=0.4):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((2 ** n, 2 ** n)) * (rng.random((2 ** n, 2 ** n)) < density)
    A[rng.integers(0, 2 ** n, 2 ** n), np.arange(2 ** n)] += 1.0     # no zero column
    return A


def _run(c, ops=None):
    st = OracleState.from_circuit(c)
    st.apply(c.ops if ops is None else ops)
    return st.export()


def test_tree_angles_reproduce_signed_vector():
    v = np.array([0.3, -0.2, 0.0, 0.5, -0.7, 0.1, 0.25, -0.05])
    th = tree_angles(v)
    amp = np.ones(8)
    for l, t in enumerate(th):
        for p in range(2 ** l):
            half = 2 ** (3 - l)
            lo = slice(p * half, p * half + half // 2)
            hi = slice(p * half + half // 2, (p + 1) * half)
            amp[lo] *= np.cos(t[p] / 2)
            amp[hi] *= np.sin(t[p] / 2)
    assert np.max(np.abs(amp - v / np.linalg.norm(v))) < 1e-15


@pytest.mark.parametrize("seed,n", [(0, 3), (1, 4)])
def test_controlled_state_preparation(seed, n):
    """U_L |k>|0>|0> = |k>|0>|phi_k>: every column, ancillas back to 0,
    amplitudes A_jk / ||A_.k|| within the angle quantisation (w = 32)."""
    A = _matrix(seed, n)
    be = block_encoding(A)
    for k in range(2 ** n):
        _, v, a = _run(circuit(be, be.ul, j=k))
        assert np.all(v[:, 0] == k) and np.all(v[:, 1] == 0) and np.all(v[:, 3] == 0)
        phi = np.zeros(2 ** n, dtype=np.complex128)
        phi[v[:, 2].astype(np.int64)] = a
        assert np.max(np.abs(phi - A[:, k] / np.linalg.norm(A[:, k]))) < 1e-8


@pytest.mark.parametrize("seed,n", [(2, 3), (3, 4)])
def test_block_encoding_top_left_block(seed, n):
    """<i|<0|<0| U_A |j>|0>|0> = A_ij / ||A||_F (Frobenius norm), for every
    column j, within the angle quantisation."""
    A = _matrix(seed, n)
    be = block_encoding(A)
    for j in range(2 ** n):
        _, v, a = _run(circuit(be, be.ua, j=j))
        assert np.all(v[:, 1] == 0) and np.all(v[:, 3] == 0)      # d and the address are clean
        top = (v[:, 2] == 0)
        col = np.zeros(2 ** n, dtype=np.complex128)
        col[v[top, 0].astype(np.int64)] = a[top]
        assert np.max(np.abs(col - A[:, j] / np.linalg.norm(A))) < 2e-8
        assert abs(np.sum(np.abs(a) ** 2) - 1.0) < 1e-12


def test_walk_step_top_block():
    """One walk step R U_A: on the ancilla-0 block R contributes +i, so
    <i,0|W|j,0> = i A_ij / ||A||_F."""
    A = _matrix(5, 3)
    be = block_encoding(A)
    W = walk_step(be)
    for j in (0, 3, 6):
        _, v, a = _run(circuit(be, W, j=j))
        top = v[:, 2] == 0
        col = np.zeros(8, dtype=np.complex128)
        col[v[top, 0].astype(np.int64)] = a[top]
        assert np.max(np.abs(col - 1j * A[:, j] / np.linalg.norm(A))) < 2e-8


def test_oracle_matches_dense_on_walk():
    """n = 2 with 6-bit angles (14 qubits): the oracle equals the dense
    checker on U_A and three walk steps from a superposition."""
    A = _matrix(7, 2, density=0.7)
    be = block_encoding(A, w=6)
    ops = np.concatenate([be.ua] + [walk_step(be)] * 3)
    amps = np.array([0.5, -0.5j, 0.5, 0.5], dtype=np.complex128)
    c = circuit(be, ops, amps=amps)
    st = OracleState.from_circuit(c)
    st.apply(ops)
    _, v, a = st.export()
    d = DenseState.from_circuit(c)
    d.apply(ops)
    dv, da = d.entries()
    o1 = np.lexsort(v.T[::-1])
    o2 = np.lexsort(dv.T[::-1])
    assert np.array_equal(v[o1], dv[o2])
    assert np.max(np.abs(a[o1] - da[o2])) < 1e-13


def test_quantisation_roundtrip():
    th = np.array([-2 * np.pi, -1.0, 0.0, 0.5, np.pi, 2 * np.pi - 1e-12])
    from paper_2503_15118_amd.qlss import quantize
    q = quantize(th, 32)
    # Ry has period 4 pi: 2 pi wraps to -2 pi, the same rotation
    d = np.mod(dequantize(q, 32) - th, 4 * np.pi)
    assert np.max(np.minimum(d, 4 * np.pi - d)) < np.pi * 2.0 ** -30
