"""ssfm_batch: independent realisations of different lengths, span counts,
launch powers and seeds in one call, against the FP64 oracle and against
one-at-a-time ssfm_forward."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from fieldcheck import check, rel
from workloads import Link, batch_config, dual_pol_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m




def entries(n_entries, steps, seed=0):
    rng = np.random.default_rng(seed)
    lengths = [1 << 12, 1 << 13, 1 << 14, 1 << 15, 1 << 16]
    out = []
    for i in range(n_entries):
        n = lengths[i % len(lengths)]
        spans = 1 + (i * 7) % 3
        p_dbm = -4 + 10 * rng.random()
        ln = Link(n_pol=2, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=spans,
                  steps_per_span=steps, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                  gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)
        a = dual_pol_field(rng, 2, n, 2, 64e9, 0.1, p_dbm)
        out.append((ln, a, 1000 + 17 * i))
    return out


def test_batch_matches_oracle_and_single_calls(ssfm):
    es = entries(13, steps=5)
    fields = [torch.from_numpy(a.astype(np.complex64)).cuda() for _, a, _ in es]
    singles = [f.clone() for f in fields]
    ssfm.ssfm_batch([ln for ln, _, _ in es], fields, [s for _, _, s in es], 0)
    torch.cuda.synchronize()
    for (ln, a, s), f, g in zip(es, fields, singles):
        plan = ssfm.Plan(ln)
        plan.forward(g, seed=s)
        torch.cuda.synchronize()
        plan.close()
        got = f.cpu().numpy().astype(np.complex128)
        want = oracle.propagate(a, ln, seed=s, realization=0)
        check(got, want, 2e-6)
        check(got, g.cpu().numpy().astype(np.complex128), 1e-6)


def test_batch_workload4_shapes_run(ssfm):
    # the workload-4 recipe (lengths 2^12..2^16, 1..10 spans, -4..+6 dBm,
    # distinct seeds) at reduced count and steps; spot-check against the oracle
    items = batch_config(n=24)
    rng = np.random.default_rng(11)
    links, fields, seeds, inputs = [], [], [], []
    for it in items:
        ln = it.link().replace(steps_per_span=4)
        a = dual_pol_field(rng, 2, ln.n_samples, 2, 64e9, 0.1, it.launch_dbm)
        links.append(ln)
        inputs.append(a)
        fields.append(torch.from_numpy(a.astype(np.complex64)).cuda())
        seeds.append(it.seed)
    ssfm.ssfm_batch(links, fields, seeds, 0)
    torch.cuda.synchronize()
    for k in (0, 5, 17):
        want = oracle.propagate(inputs[k], links[k], seed=seeds[k], realization=0)
        check(fields[k].cpu().numpy().astype(np.complex128), want, 2e-6)


def test_batch_rejects_invalid_entries(ssfm):
    ln = Link(n_pol=2, n_samples=1000, sample_rate_hz=128e9, span_km=80.0, n_spans=1,
              steps_per_span=2, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
              gamma_per_w_km=1.3)
    f = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
    with pytest.raises(ssfm.SsfmError) as e:
        ssfm.ssfm_batch([ln], [f], [1], 0)
    assert e.value.status == ssfm.SSFM_EINVAL


def test_batch_groups_concurrent_bitwise(ssfm):
    # more link groups than worker streams (sizes x fibre parameters, both
    # paths): every entry equals its single ssfm_forward call bit for bit, and
    # two batch calls agree bit for bit
    rng = np.random.default_rng(23)
    links, inputs, seeds = [], [], []
    for i in range(14):
        n = [1 << 12, 1 << 13, 1 << 14, 1 << 15][i % 4]
        ln = Link(n_pol=2, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=1 + i % 3,
                  steps_per_span=3, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                  gamma_per_w_km=1.3 if i < 7 else 1.1, edfa_gain_db=16.0, edfa_nf_db=5.0,
                  ase=True)
        links.append(ln)
        inputs.append(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 2.0))
        seeds.append(300 + i)
    runs = []
    for _ in range(2):
        fields = [torch.from_numpy(a.astype(np.complex64)).cuda() for a in inputs]
        ssfm.ssfm_batch(links, fields, seeds, 0)
        torch.cuda.synchronize()
        runs.append([f.cpu().numpy() for f in fields])
    for k, (ln, a, s) in enumerate(zip(links, inputs, seeds)):
        assert np.array_equal(runs[0][k], runs[1][k]), k
        g = torch.from_numpy(a.astype(np.complex64)).cuda()
        plan = ssfm.Plan(ln)
        plan.forward(g, seed=s)
        torch.cuda.synchronize()
        plan.close()
        assert np.array_equal(runs[0][k], g.cpu().numpy()), (k, ln.n_samples)


def test_batch_workload4_full_size(ssfm):
    # workload 4 as stated: 256 realisations, 50 steps per span, 1..10 spans,
    # lengths 2^12..2^16.  Per length group, the entry with the fewest spans
    # (it runs only in the group's first segment, the widest: seeded wide
    # tiles on the four-step lengths) and the one with the most (every
    # segment, down to the narrow tiles of the last ones) against the oracle
    items = batch_config(256)
    rng = np.random.default_rng(20250703 + 44)
    links = [it.link() for it in items]
    assert all(ln.steps_per_span == 50 for ln in links)
    inputs = [dual_pol_field(rng, 2, ln.n_samples, 2, 64e9, 0.1, it.launch_dbm)
              for it, ln in zip(items, links)]
    seeds = [it.seed for it in items]
    fields = [torch.from_numpy(a.astype(np.complex64)).cuda() for a in inputs]
    ssfm.ssfm_batch(links, fields, seeds, 0)
    torch.cuda.synchronize()
    picked = []
    for n in sorted({ln.n_samples for ln in links}):
        idx = [i for i, ln in enumerate(links) if ln.n_samples == n]
        picked += sorted({min(idx, key=lambda i: links[i].n_spans),
                          max(idx, key=lambda i: links[i].n_spans)})
    assert len(picked) >= 9
    for k in picked:
        print(f"entry {k}: n={links[k].n_samples} spans={links[k].n_spans}", flush=True)
        want = oracle.propagate(inputs[k], links[k], seed=seeds[k], realization=0)
        check(fields[k].cpu().numpy().astype(np.complex128), want, 2e-6, what=f"entry {k}")


def test_batch_graph_replay_is_bitwise(ssfm):
    # the same call repeated: the first runs directly, the second captures
    # the launch sequence (after measuring launch shapes for every group's
    # active counts) and launches the graph, later ones replay it.  Every
    # call restarts from the same inputs (copied in by eager work between
    # the calls); all outputs equal the first, bit for bit, and the oracle.
    # A different call in between drops the graph; the next repeats capture
    # again.
    es = entries(11, steps=4, seed=5)
    links = [ln for ln, _, _ in es]
    seeds = [s for _, _, s in es]
    inputs = [torch.from_numpy(a.astype(np.complex64)).cuda() for _, a, _ in es]
    fields = [x.clone() for x in inputs]
    other = entries(3, steps=2, seed=6)
    other_fields = [torch.from_numpy(a.astype(np.complex64)).cuda() for _, a, _ in other]
    outs = []
    for call in range(7):
        for f, x in zip(fields, inputs):
            f.copy_(x)
        if call == 4:
            # a different call: the replay graph is dropped
            ssfm.ssfm_batch([ln for ln, _, _ in other], other_fields, [s for _, _, s in other], 0)
        ssfm.ssfm_batch(links, fields, seeds, 0)
        torch.cuda.synchronize()
        outs.append([f.cpu().numpy() for f in fields])
        print(f"call {call} done", flush=True)
    for call in range(1, len(outs)):
        for k in range(len(es)):
            assert np.array_equal(outs[call][k], outs[0][k]), (call, k)
    for k in (0, 4, 7):
        ln, a, s = es[k]
        want = oracle.propagate(a, ln, seed=s, realization=0)
        check(outs[-1][k].astype(np.complex128), want, 2e-6, what=f"entry {k}")
