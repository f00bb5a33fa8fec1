"""Batched permanents + gradients of real matrices (the one-component form of
the batched launch) against the oracle, the complex plan and the
single-matrix gradient."""
import time
from fractions import Fraction

import numpy as np
import pytest
import torch

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
U = 2.0 ** -53


def signed_batch(ks, seed):
    """Real matrices with entries uniform in [-1, 1) (cancellation in every sum)."""
    rng = np.random.default_rng(seed)
    return [2.0 * rng.random((k, k)) - 1.0 for k in ks]


def run(mats, want_grad=True, use_graph=True, autotune=False, real=True):
    ks, offs, data = W.pack(mats)
    if not real:
        data = data.astype(np.complex128)
    d = torch.from_numpy(data).to(DEV)
    with api.BatchedPlan(ks, offs, want_grad=want_grad, real=real) as plan:
        if autotune:
            plan.autotune(d)
        out, grad = plan.run(d, use_graph=use_graph)
        info = plan.info()
        o = out.cpu().numpy()
        g = None
        if grad is not None:
            gh = grad.cpu().numpy()
            g = [gh[off:off + k * k].reshape(k, k) for k, off in zip(ks, offs)]
    return o, g, info


def loo_abs_sums(a):
    """S_i = sum over the 2^(k-1) Gray-walk vectors x = a_{k-1}/2 + sum_j<k-1
    a_j s_j (s_j = +-1/2) of prod_{l != i} |x_l|: the absolute sum behind
    row i of the gradient sweep (brute force, small k)."""
    k = a.shape[0]
    if k == 1:
        return np.ones(1)
    s = np.array([[0.5 if (g >> j) & 1 else -0.5 for j in range(k - 1)] + [0.5]
                  for g in range(1 << (k - 1))])
    x = np.abs(s @ a.T)  # (subsets, rows)
    out = np.zeros(k)
    for i in range(k):
        out[i] = np.sum(np.prod(np.delete(x, i, axis=1), axis=1))
    return out


KS = [1, 2, 3, 4, 5, 7, 8, 11, 12, 13, 16, 17, 19, 20, 23, 24, 25, 27]


def test_real_mixed_orders_vs_oracle(oracle):
    mats = signed_batch(KS, 101)
    out, g, _ = run(mats)
    for m, a in enumerate(mats):
        k = a.shape[0]
        want, r = oracle.ryser(a, with_abs=True)
        # the same gate as the complex batch: 1e-13 (about 900 u) times R(A),
        # the absolute sum of the Ryser terms
        assert abs(out[m] - want) <= 1e-13 * r + 1e-300, (m, out[m], want, r)
        if k <= 12:
            gm = oracle.grad_minors(a)
            srow = loo_abs_sums(a)
            for i in range(k):
                for j in range(k):
                    assert abs(g[m][i, j] - gm[i, j]) <= 1e-13 * srow[i] + 1e-300, (m, i, j)


def test_real_plan_matches_complex_plan(oracle):
    # the same real matrices through the complex kernels (imaginary parts 0)
    mats = signed_batch([6, 9, 14, 18, 22, 26], 111)
    out_r, g_r, _ = run(mats)
    out_c, g_c, _ = run(mats, real=False)
    assert np.all(out_c.imag == 0.0)
    for m, a in enumerate(mats):
        _, r = oracle.ryser(a, with_abs=True)
        assert abs(out_r[m] - out_c[m].real) <= 1e-13 * r, m
        assert np.all(g_c[m].imag == 0.0)
        scale = np.max(np.abs(g_c[m]))
        assert np.max(np.abs(g_r[m] - g_c[m].real)) <= 1e-11 * scale, m


def test_real_matches_single_matrix_grad():
    # orders in every kernel group, up to 32, against perm_grad (real)
    mats = signed_batch([11, 15, 18, 21, 23, 28], 121) + [W.uniform(32, 1700)]
    out, g, _ = run(mats)
    for m, a in enumerate(mats):
        p, gs = api.perm_grad(torch.from_numpy(np.ascontiguousarray(a)).to(DEV))
        gs = gs.cpu().numpy()
        scale = np.max(np.abs(gs))
        assert abs(out[m] - p.item()) <= 1e-12 * abs(p.item()) + 1e-13 * scale, m
        assert np.max(np.abs(g[m] - gs)) <= 1e-11 * scale, m
    # Laplace's identity along every row and column of the 32 x 32 matrix
    a = mats[-1]
    for i in range(32):
        assert abs(np.dot(a[i], g[-1][i]) - out[-1]) <= 1e-10 * abs(out[-1]), i
        assert abs(np.dot(a[:, i], g[-1][:, i]) - out[-1]) <= 1e-10 * abs(out[-1]), i


def test_real_forward_only_and_graph_replays():
    mats = signed_batch([8, 13, 17, 22, 24, 6, 30], 131)
    ks, offs, data = W.pack(mats)
    d = torch.from_numpy(data).to(DEV)
    with api.BatchedPlan(ks, offs, want_grad=True, real=True) as plan:
        out_e, grad_e = plan.run(d, use_graph=False)
        out_e, grad_e = out_e.clone(), grad_e.clone()
        out, grad = plan.outputs(d)
        for rep in range(3):
            out.zero_()
            grad.zero_()
            plan.run(d, out=out, grad=grad, use_graph=True)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(out, out_e), rep
            assert torch.equal(grad, grad_e), rep
            del junk
    with api.BatchedPlan(ks, offs, want_grad=False, real=True) as plan:
        out_f, g = plan.run(d)
        assert g is None
        assert torch.allclose(out_f, out_e, rtol=1e-12, atol=0)
        with pytest.raises(ValueError):
            plan.run(d.to(torch.complex128))


def test_real_autotune_kept_apart_from_complex():
    # orders up to 24 (the groups of orders 1..16 and 17..24 in the graph, as
    # in the bench's batch): autotuning with the kernel of orders 25..32
    # forked beside them is kept off the GPU until a stall seen there is
    # explained
    mats = signed_batch([10, 16, 21, 23, 24], 141)
    out0, g0, _ = run(mats)
    out1, g1, info = run(mats, autotune=True)
    assert info["log2_chunk"] in (8, 10, 12)
    for m, a in enumerate(mats):
        # scale: sum_j |a_0j G_0j|, the absolute terms of perm's expansion along row 0
        assert abs(out1[m] - out0[m]) <= 1e-12 * np.sum(np.abs(a[0] * g0[m][0]))
        assert np.max(np.abs(g1[m] - g0[m])) <= 1e-11 * np.max(np.abs(g0[m]))
    ks, offs, data = W.pack(mats)
    with api.BatchedPlan(ks, offs, want_grad=True, real=True) as plan:
        assert plan.info()["tuned_from_cache"]
        t0 = time.perf_counter()
        plan.autotune(torch.from_numpy(data).to(DEV))
        assert time.perf_counter() - t0 < 0.05
    # a complex plan with the same orders keeps its own tuning
    with api.BatchedPlan(ks, offs, want_grad=True) as plan:
        assert not plan.info()["tuned_from_cache"]


def test_weighted_sum_f64_exact_order():
    # sum_m w_m p_m in double-double: within one final rounding of the exact
    # sum, for values spread over 60 binades of which a third cancel in pairs
    rng = np.random.default_rng(151)
    p = rng.standard_normal(1000) * 2.0 ** rng.integers(-30, 30, 1000)
    w = rng.standard_normal(1000)
    p = np.concatenate([p, -p[:500]])
    w = np.concatenate([w, w[:500]])
    want = float(sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(w, p)))
    from paper_2502_16577_amd import _native as N
    wt, pt = torch.from_numpy(w).to(DEV), torch.from_numpy(p).to(DEV)
    out = torch.zeros((), dtype=torch.float64, device=DEV)
    N.check(N.lib().perm_weighted_sum_f64(len(p), wt.data_ptr(), pt.data_ptr(), out.data_ptr(),
                                          api._stream(DEV)), "perm_weighted_sum_f64")
    got = out.item()
    scale = float(np.sum(np.abs(w * p)))
    assert abs(got - want) <= 4 * U * abs(want) + 1e3 * U * U * scale, (got, want)


@pytest.mark.parametrize("real", [True, False])
def test_weighted_sum_keeps_product_rounding_errors(real):
    # pairs w * p and 1 * (-fl(w p)): the exact sum is the sum of the
    # products' rounding errors alone, which the double-double sum keeps (an
    # FP64 sum returns noise; an error term counted twice doubles it)
    from paper_2502_16577_amd import _native as N
    rng = np.random.default_rng(161)
    w = 1.0 + rng.random(400)
    p = rng.standard_normal(400)
    q = -(w * p)
    wts = np.concatenate([w, np.ones(400)])
    vals = np.concatenate([p, q])
    exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(wts, vals))
    assert exact != 0
    wt = torch.from_numpy(wts).to(DEV)
    if real:
        pt = torch.from_numpy(vals).to(DEV)
        out = torch.zeros((), dtype=torch.float64, device=DEV)
        fn = N.lib().perm_weighted_sum_f64
    else:  # the same values as real parts, their negatives as imaginary parts
        pt = torch.from_numpy(vals - 1j * vals).to(DEV)
        out = torch.zeros((), dtype=torch.complex128, device=DEV)
        fn = N.lib().perm_weighted_sum
    N.check(fn(len(vals), wt.data_ptr(), pt.data_ptr(), out.data_ptr(), api._stream(DEV)),
            "weighted sum")
    got = complex(out.item())
    assert abs(Fraction(got.real) - exact) <= Fraction(1, 10 ** 12) * abs(exact), (got, float(exact))
    if not real:
        assert abs(Fraction(got.imag) + exact) <= Fraction(1, 10 ** 12) * abs(exact), (got, float(exact))
