"""The planner's register program, interpreted on the CPU, reproduces the
dense oracle: this checks the plan (host logic) independently of the kernels."""

import numpy as np
import pytest

import synth
from oracle import dense


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    return m


def _interpret(ops, wg, fac, l2, gates_u, gates_v):
    """Evaluate the program with numpy (register bit i = axis weight 2^i)."""
    s = len(gates_u)
    b = 0
    reg = np.ones(1, dtype=np.complex128)

    def mat(k):
        m = np.eye(4, dtype=np.complex128)
        first, cnt = wg[k]
        for f in fac[first:first + cnt]:
            g = gates_v[f] if f < s else np.conj(gates_u[2 * s - 1 - f]).T
            m = g @ m
        return m

    for op in ops:
        t, p, q = int(op["type"]) & 3, int(op["p"]), int(op["q"])
        if t == 0:
            m = mat(int(op["arg"]))
            # R[(y_in, y_out), (x_in, x_out)] = M[2 x_out + y_out, 2 x_in + y_in]
            r = np.empty((2, 2, 2, 2), dtype=np.complex128)
            for yi in range(2):
                for yo in range(2):
                    for xi in range(2):
                        for xo in range(2):
                            r[yi, yo, xi, xo] = m[2 * xo + yo, 2 * xi + yi]
            t_ = reg.reshape([2] * b)              # axis k <-> bit b-1-k
            ap, aq = b - 1 - p, b - 1 - q
            t_ = np.moveaxis(t_, (ap, aq), (0, 1))
            t_ = np.einsum("abcd,cd...->ab...", r, t_)
            reg = np.moveaxis(t_, (0, 1), (ap, aq)).reshape(-1)
        elif t == 1:
            new = np.zeros(4 * reg.size, dtype=np.complex128)
            new[: reg.size] = reg
            new[3 * reg.size:] = reg
            reg = new
            b += 2
        elif t == 2:
            t_ = reg.reshape([2] * b)
            ap, aq = b - 1 - p, b - 1 - q
            t_ = np.trace(t_, axis1=ap, axis2=aq)
            reg = t_.reshape(-1)
            b -= 2
        assert b == int(op["bits"])
    assert b == 0
    return complex(reg[0]) * 2.0 ** l2


def _circ(n, bonds, gates):
    return {"ansatz": 1, "n": n, "gates": [(int(bb), g) for bb, g in zip(bonds, gates)]}


def test_program_matches_dense_random_gates(fp):
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(2, 8))
        s = int(rng.integers(1, 16))
        bu = rng.integers(0, n - 1, s)
        bv = rng.integers(0, n - 1, s)
        gu = synth.complex_gaussian(1000 + trial, (s, 4, 4)) * 0.5
        gv = synth.complex_gaussian(2000 + trial, (s, 4, 4)) * 0.5
        ops, wg, fac, l2 = fp.fp_plan_program_host(n, bu, bv)
        got = _interpret(ops, wg, fac, l2, gu, gv)
        want = dense.trace_pair(_circ(n, bu, gu), _circ(n, bv, gv))
        assert abs(got - want) <= 1e-10 * max(1.0, abs(want)), (n, list(bu), list(bv), got, want)


def test_program_brickwork_layout(fp):
    from oracle.sampler import brickwork_layout
    for n, d in [(4, 1), (5, 2), (6, 3), (6, 4)]:
        bonds = brickwork_layout(n, d)
        s = len(bonds)
        gu = synth.complex_gaussian(77 + d, (s, 4, 4)) * 0.5
        gv = synth.complex_gaussian(88 + d, (s, 4, 4)) * 0.5
        ops, wg, fac, l2 = fp.fp_plan_program_host(n, bonds, bonds)
        got = _interpret(ops, wg, fac, l2, gu, gv)
        want = dense.trace_pair(_circ(n, bonds, gu), _circ(n, bonds, gv))
        assert abs(got - want) <= 1e-10 * max(1.0, abs(want))
