"""GPU adjoint (ssfm_adjoint through the C ABI, and the autograd wrapper)
against the FP64 oracle's adjoint, whose pins are in test_oracle_adjoint."""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from fieldcheck import check, rel
from workloads import CONFIGS, Link, dual_pol_field, make_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m




def link(n_pol, n, spans, steps, **kw):
    base = dict(n_pol=n_pol, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=spans,
                steps_per_span=steps, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)
    base.update(kw)
    return Link(**base)


def gpu_adjoint(ssfm, x, g, ln, seed, state_bytes=0):
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).cuda()
    gt = torch.from_numpy(np.ascontiguousarray(g, dtype=np.complex64)).cuda()
    plan = ssfm.Plan(ln)
    try:
        if state_bytes:
            plan.set_state_memory(state_bytes)
        plan.adjoint(xt, gt, seed=seed)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return gt.cpu().numpy().astype(np.complex128), xt.cpu().numpy()


@pytest.mark.parametrize("n,n_pol", [(1 << 14, 2), (1 << 14, 1), (1 << 16, 2), (1 << 18, 2)])
def test_adjoint_matches_oracle(ssfm, n, n_pol):
    print(f"case n={n} n_pol={n_pol}", flush=True)
    rng = np.random.default_rng(n + n_pol)
    ln = link(n_pol, n, spans=2, steps=5)
    b = 2
    x = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
    g = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
    got, x_after = gpu_adjoint(ssfm, x, g, ln, seed=21)
    assert np.array_equal(x_after, x.astype(np.complex64))  # input untouched
    for r in range(b):
        want = oracle.adjoint(x[r], g[r], ln, seed=21, realization=r)
        check(got[r], want, 1e-5)


def test_adjoint_workload2_full_link(ssfm):
    w = CONFIGS[2]
    x = make_field(w)
    rng = np.random.default_rng(5)
    g = dual_pol_field(rng, 2, w.link.n_samples, 2, 64e9, 0.1, 0.0)
    got, _ = gpu_adjoint(ssfm, x[None], g[None], w.link, seed=w.ase_seed)
    want = oracle.adjoint(x, g, w.link, seed=w.ase_seed)
    err = rel(got[0], want)
    print(f"workload2 adjoint rel_err={err:.3e}", flush=True)
    assert err < 1e-5


def test_adjoint_workload2_bench_configuration(ssfm):
    # the benchmarked adjoint: 512 realisations without kept spans, the
    # forward pass in two 256-realisation chunks, the reverse sweep in four
    # chunks of 128, every chunk as two concurrent parts; sampled
    # realisations on both sides of chunk and part boundaries against the
    # oracle's adjoint, one by one
    w = CONFIGS[2]
    batch = 512
    host = np.stack([make_field(w, seed=w.symbol_seed + i) for i in range(8)])
    rng = np.random.default_rng(512)
    gh = np.stack([dual_pol_field(rng, 2, w.link.n_samples, 2, 64e9, 0.1, 0.0) for _ in range(8)])
    x = np.tile(host, (batch // 8, 1, 1))
    g = np.tile(gh, (batch // 8, 1, 1))
    got, _ = gpu_adjoint(ssfm, x, g, w.link, seed=w.ase_seed)
    for r in (63, 64, 511):
        print(f"workload2 adjoint batch 512: realisation {r}", flush=True)
        want = oracle.adjoint(x[r], g[r], w.link, seed=w.ase_seed, realization=r)
        check(got[r], want, 1e-5, what=f"realisation {r}")


def test_autograd_mse_gradient(ssfm):
    n = 1 << 14
    ln = link(2, n, spans=2, steps=4)
    rng = np.random.default_rng(17)
    x0 = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 4.0)
    target = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 4.0)
    plan = ssfm.Plan(ln)
    x = torch.from_numpy(x0.astype(np.complex64))[None].cuda().requires_grad_(True)
    t = torch.from_numpy(target.astype(np.complex64))[None].cuda()
    y = ssfm.propagate(x, plan, seed=3)
    loss = torch.mean(torch.abs(y - t) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    # dL/dy* = (y - t) / numel; PyTorch's complex gradient is 2 dL/dz*.  The
    # oracle's cotangent is formed from its own output y (no oracle input
    # comes from the GPU); the two outputs differ by ~1e-6
    y_np = oracle.propagate(x0, ln, seed=3)
    gy = (y_np - target) / y_np.size
    want = 2 * oracle.adjoint(x0, gy, ln, seed=3)
    got = x.grad.detach().cpu().numpy().astype(np.complex128)[0]
    check(got, want, 1e-5)
    plan.close()


# ---------------------------------------------------------------------------
# LDS-resident path (n <= 2^13): one launch, span checkpoints, each span
# recomputed from its checkpoint before its reverse sweep
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,n_pol", [(64, 1), (64, 2), (512, 2), (2048, 1), (4096, 1),
                                     (4096, 2), (8192, 1), (8192, 2)])
def test_adjoint_lds_path_matches_oracle(ssfm, n, n_pol):
    print(f"case n={n} n_pol={n_pol}", flush=True)
    rng = np.random.default_rng(3 * n + n_pol)
    ln = link(n_pol, n, spans=3, steps=4)
    b = 2
    x = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
    g = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
    got, x_after = gpu_adjoint(ssfm, x, g, ln, seed=17)
    assert np.array_equal(x_after, x.astype(np.complex64))  # input untouched
    for r in range(b):
        want = oracle.adjoint(x[r], g[r], ln, seed=17, realization=r)
        check(got[r], want, 1e-5, what=f"realisation {r}")


def test_adjoint_workload1(ssfm):
    # NLSE, 4096 samples, one 80 km span in 80 steps, no amplifier
    w = CONFIGS[1]
    ln = w.link
    x = make_field(w, seed=w.symbol_seed)[None]
    rng = np.random.default_rng(11)
    g = dual_pol_field(rng, 1, ln.n_samples, 2, 32e9, 0.1, 0.0)[None]
    got, _ = gpu_adjoint(ssfm, x, g, ln, seed=0)
    want = oracle.adjoint(x[0], g[0], ln, seed=0)
    check(got[0], want, 1e-5)


def test_adjoint_lds_path_large_nonlinear_phase(ssfm):
    # several rad per step: the general phasor routine in both passes
    n = 2048
    ln = link(2, n, spans=2, steps=3, span_km=60.0)
    rng = np.random.default_rng(12)
    x = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 18.0)[None]
    g = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0)[None]
    got, _ = gpu_adjoint(ssfm, x, g, ln, seed=4)
    want = oracle.adjoint(x[0], g[0], ln, seed=4)
    check(got[0], want, 1e-5)


def test_autograd_lds_path(ssfm):
    n = 4096
    ln = link(2, n, spans=2, steps=3)
    rng = np.random.default_rng(13)
    x0 = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 4.0)
    target = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 4.0)
    plan = ssfm.Plan(ln)
    try:
        x = torch.from_numpy(x0.astype(np.complex64))[None].cuda().requires_grad_(True)
        y = ssfm.propagate(x, plan, seed=8)
        loss = (y - torch.from_numpy(target.astype(np.complex64)).cuda()).abs().pow(2).sum()
        loss.backward()
        torch.cuda.synchronize()
        y_np = oracle.propagate(x0, ln, seed=8)
        want = 2 * oracle.adjoint(x0, (y_np - target), ln, seed=8)
        got = x.grad.detach().cpu().numpy().astype(np.complex128)[0]
        check(got, want, 1e-5)
    finally:
        plan.close()


@pytest.mark.parametrize("kept", [False, True])
@pytest.mark.parametrize("n,n_pol", [(1 << 14, 2), (1 << 15, 1)])
def test_adjoint_large_nonlinear_phase(ssfm, n, n_pol, kept):
    # 18 dBm over 20 km steps: per-step phases of several rad on most samples
    print(f"case n={n} n_pol={n_pol} kept={kept}", flush=True)
    rng = np.random.default_rng(n + n_pol)
    ln = link(n_pol, n, spans=1, steps=4)
    x = dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 18.0)
    g = dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 0.0)
    budget = 4 * n_pol * n * 8 if kept else 0
    got, _ = gpu_adjoint(ssfm, x[None], g[None], ln, seed=3, state_bytes=budget)
    want = oracle.adjoint(x, g, ln, seed=3)
    check(got[0], want, 1e-5)


# ---------------------------------------------------------------------------
# kept spans: the forward pass stores the nonlinear-step inputs of the last
# K spans (K set by the state budget) and their reverse sweep carries the
# cotangent alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,n_pol,spans,kept", [(1 << 16, 2, 3, 3), (1 << 16, 2, 3, 1),
                                                (1 << 14, 1, 2, 2), (1 << 15, 2, 2, 1),
                                                (1 << 18, 2, 2, 2)])
def test_adjoint_kept_spans_match_oracle(ssfm, n, n_pol, spans, kept):
    print(f"case n={n} n_pol={n_pol} spans={spans} kept={kept}", flush=True)
    rng = np.random.default_rng(3 * n + n_pol + spans)
    steps, b = 5, 2
    ln = link(n_pol, n, spans=spans, steps=steps)
    x = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
    g = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
    per_span = steps * b * n_pol * n * 8
    got, x_after = gpu_adjoint(ssfm, x, g, ln, seed=9, state_bytes=kept * per_span + per_span // 2)
    assert np.array_equal(x_after, x.astype(np.complex64))
    rebuilt, _ = gpu_adjoint(ssfm, x, g, ln, seed=9)
    for r in range(b):
        want = oracle.adjoint(x[r], g[r], ln, seed=9, realization=r)
        check(got[r], want, 1e-5)
        check(got[r], rebuilt[r], 5e-6)


def test_adjoint_state_budget_reuse_and_release(ssfm):
    # the store is kept by the plan across calls; a zero budget releases it
    # and the next call is the reconstructing sweep again, bit for bit
    n, steps = 1 << 15, 4
    ln = link(2, n, spans=2, steps=steps)
    rng = np.random.default_rng(41)
    x = torch.from_numpy(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0).astype(np.complex64))[None].cuda()
    g0 = torch.from_numpy(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0).astype(np.complex64))[None].cuda()
    plan = ssfm.Plan(ln)
    try:
        plain = plan.adjoint(x, g0.clone())
        plan.set_state_memory(2 * steps * 2 * n * 8)
        kept1 = plan.adjoint(x, g0.clone())
        kept2 = plan.adjoint(x, g0.clone())
        plan.set_state_memory(0)
        again = plan.adjoint(x, g0.clone())
        torch.cuda.synchronize()
        assert torch.equal(kept1, kept2)
        assert torch.equal(plain, again)
        assert not torch.equal(plain, kept1)  # a different rounding path
        a = plain.cpu().numpy().astype(np.complex128)
        k = kept1.cpu().numpy().astype(np.complex128)
        check(k, a, 5e-6)
    finally:
        plan.close()


@pytest.mark.parametrize("kept,parts", [(0, 2), (1, 2), (0, 3)])
def test_adjoint_two_stream_split_is_bitwise(ssfm, kept, parts):
    # the adjoint of concurrent parts (each on its share of the workspace)
    # against the single-stream call: the same bits
    print(f"case kept={kept} parts={parts}", flush=True)
    n, steps, b = 1 << 15, 3, 5
    ln = link(2, n, spans=2, steps=steps)
    rng = np.random.default_rng(77 + kept)
    x = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
    g = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
    xt = torch.from_numpy(x.astype(np.complex64)).cuda()
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    plan = ssfm.Plan(ln)
    try:
        plan.set_state_memory(kept * steps * b * 2 * n * 8)
        out = {}
        for streams in (parts, 1):
            plan.set_forward_streams(streams)
            out[streams] = plan.adjoint(xt, gt.clone(), seed=6)
        torch.cuda.synchronize()
        assert torch.equal(out[1], out[parts])
        got = out[parts].cpu().numpy().astype(np.complex128)
    finally:
        plan.close()
    for r in (0, b - 1):
        want = oracle.adjoint(x[r], g[r], ln, seed=6, realization=r)
        check(got[r], want, 1e-5)


def test_adjoint_calls_on_two_streams(ssfm):
    # two adjoint calls on one plan, issued back to back on two streams: the
    # plan serialises them on the device (they share its workspace), so each
    # returns what it returns alone
    n, steps = 1 << 15, 3
    ln = link(2, n, spans=2, steps=steps)
    rng = np.random.default_rng(55)
    xs = [torch.from_numpy(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0)
                           .astype(np.complex64))[None].cuda() for _ in range(2)]
    gs = [torch.from_numpy(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0)
                           .astype(np.complex64))[None].cuda() for _ in range(2)]
    plan = ssfm.Plan(ln)
    try:
        alone = []
        for x, g in zip(xs, gs):
            alone.append(plan.adjoint(x, g.clone(), seed=3))
            torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        outs = [g.clone() for g in gs]
        torch.cuda.synchronize()
        plan.adjoint(xs[0], outs[0], seed=3, stream=s1)
        plan.adjoint(xs[1], outs[1], seed=3, stream=s2)
        torch.cuda.synchronize()
        for a, o in zip(alone, outs):
            assert torch.equal(a, o)
    finally:
        plan.close()


def test_adjoint_state_store_refused_keeps_fewer_spans(ssfm, monkeypatch):
    # the budget holds 3 spans but the device (fault injection) refuses a
    # store of more than one: the call keeps one span and the result is the
    # oracle's adjoint, close to the reconstructing sweep's
    n, steps, spans = 1 << 14, 3, 3
    ln = link(2, n, spans=spans, steps=steps)
    rng = np.random.default_rng(66)
    x = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0)[None]
    g = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0)[None]
    monkeypatch.setenv("SSFM_FAIL_STATE_ALLOC", "1")
    got, _ = gpu_adjoint(ssfm, x, g, ln, seed=2, state_bytes=spans * steps * 2 * n * 8)
    monkeypatch.delenv("SSFM_FAIL_STATE_ALLOC")
    rebuilt, _ = gpu_adjoint(ssfm, x, g, ln, seed=2)
    want = oracle.adjoint(x[0], g[0], ln, seed=2, realization=0)
    check(got[0], want, 1e-5)
    check(got[0], rebuilt[0], 5e-6)
    assert not np.array_equal(got, rebuilt)  # a kept span took the stored path
