"""GPU checks of the batched sweep (one persistent kernel in a captured hipGraph).

The sweep draws the same channel as awgn_sample (seed_i, offset = s * N_i) and computes
the GMI loss from the subset sums directly (log2(S0 + S1) - log2(S_sent) per bit, the
same quantity as softplus of the LLR); compared with the per-instance path
awgn_sample -> llr_exact -> gmi_reduce the difference is FP32 rounding only.  Both paths
take base-2 logarithms of sums scaled by 2^100 (|log2| up to about 130, so a few 2^-24
of 130 per logarithm, two per bit term) and the hardware logarithm need not round
symmetrically, so the averages can differ by a few 1e-5; the bar is the parity bar,
|dGMI| <= 1e-4 bit, which each path also meets against the FP64 oracle.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd as m
    return m


def make_instances(specs, seed=5):
    inst, host = [], []
    for k, (M, D, N) in enumerate(specs):
        X, labels = synth.gaussian_constellation(M, D, seed * 100 + k)
        labels = synth.random_labels(M, seed + k)
        Xd = torch.from_numpy(X).cuda()
        ld = torch.from_numpy(labels.astype(np.int32)).cuda()
        inst.append((Xd, ld, N, 1000 + k))
        host.append((X, labels))
    return inst, host


def per_instance_gmi(inst, sigma2):
    out = np.zeros(sigma2.shape)
    for i, (Xd, ld, N, seed) in enumerate(inst):
        for s in range(sigma2.shape[1]):
            tx, y = md().awgn_sample(Xd, seed, s * N, N, math.sqrt(sigma2[i, s]))
            L = md().llr_exact(Xd, ld, y, sigma2[i, s])
            out[i, s] = md().gmi_reduce(L, tx, ld)[0].item()
    return out


SPECS = [(16, 2, 3001), (64, 4, 5000), (256, 8, 4000), (1024, 2, 2500), (4096, 8, 1200), (32, 8, 777),
         (128, 4, 1), (2048, 8, 3000)]


def sigma2_grid(host, snrs):
    return np.array([[synth.sigma2_from_snr_db(X, s) for s in snrs] for X, _ in host])


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_sweep_matches_per_instance_path(variant):
    inst, host = make_instances(SPECS)
    s2 = sigma2_grid(host, [2.0, 7.0, 12.0])
    plan = md().SweepPlan(inst, s2, variant=variant)
    g = plan.run().cpu().numpy()
    ref = per_instance_gmi(inst, s2)
    assert np.all(np.isfinite(g))
    np.testing.assert_allclose(g, ref, atol=1e-4, rtol=0)
    plan.close()


@pytest.mark.parametrize("variant", [0, 3, 4])
def test_every_channel_dimension_matches_the_per_instance_path(variant):
    """The sweep kernels draw the channel with the dimension fixed at compile time (one
    instantiation per D), the per-instance path with awgn_sample's run-time D: every
    dimension the sweep takes besides 2, 4 and 8 (1, 3, 5, 6, 7), through the matrix-core
    kernel (variant 0: two symbol blocks per wavefront; 3: one block, both lane halves
    drawing) and the vector kernel (variant 4, M <= 64), gives the per-instance GMI."""
    specs = [(64, 1, 1500), (256, 3, 1200), (1024, 5, 700), (32, 6, 1100), (128, 7, 900), (64, 5, 1300),
             (16, 7, 1000), (512, 6, 800)]
    inst, host = make_instances(specs, seed=71)
    s2 = sigma2_grid(host, [3.0, 11.0])
    plan = md().SweepPlan(inst, s2, variant=variant)
    g = plan.run().cpu().numpy()
    ref = per_instance_gmi(inst, s2)
    assert np.all(np.isfinite(g))
    np.testing.assert_allclose(g, ref, atol=1e-4, rtol=0)
    plan.close()


def test_sweep_against_oracle():
    inst, host = make_instances([(64, 4, 20000), (256, 2, 8000)], seed=9)
    s2 = sigma2_grid(host, [4.0, 10.0])
    plan = md().SweepPlan(inst, s2, variant=0)
    g = plan.run().cpu().numpy()
    for i, (X, labels) in enumerate(host):
        for s in range(2):
            N, seed = inst[i][2], inst[i][3]
            tx, y = oracle.awgn(X, seed, s * N, N, math.sqrt(s2[i, s]))
            gr, _, _ = oracle.gmi(oracle.llr_exact(X, labels, y, s2[i, s]), tx, labels)
            assert abs(g[i, s] - gr) <= 1e-4, (i, s, g[i, s], gr)


def test_graph_replays_equal_eager_and_are_deterministic():
    inst, host = make_instances(SPECS[:5], seed=3)
    s2 = sigma2_grid(host, [3.0, 9.0])
    plan = md().SweepPlan(inst, s2, variant=1)
    eager = plan.run(use_graph=False).cpu().numpy()
    for _ in range(3):
        # unrelated eager work between replays
        md().llr_exact(inst[1][0], inst[1][1], torch.zeros((100, 4), device="cuda"), 0.3)
        torch.cuda.synchronize()
        g = plan.run(use_graph=True).cpu().numpy()
        assert np.array_equal(g, eager)


def test_autotuned_plan_and_limits():
    inst, host = make_instances(SPECS[:4], seed=4)
    s2 = sigma2_grid(host, [5.0])
    plan = md().SweepPlan(inst, s2, variant=-1)
    assert plan.shape in [(8, 2, 1), (8, 2, 4), (16, 1, 1), (16, 1, 4), (4, 1, 4)]
    ref = per_instance_gmi(inst, s2)
    np.testing.assert_allclose(plan.run().cpu().numpy(), ref, atol=1e-4, rtol=0)
    X, labels = synth.gaussian_constellation(8, 2, 1)
    bad = [(torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda(), 100, 1)]
    with pytest.raises(md().MdemapError) as e:
        md().SweepPlan(bad, np.array([[0.1]]))
    assert e.value.status == -8
    X, labels = synth.gaussian_constellation(64, 12, 1)
    bad = [(torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda(), 100, 1)]
    with pytest.raises(md().MdemapError):
        md().SweepPlan(bad, np.array([[0.1]]))


def oracle_gmi(host, inst, s2, i, s):
    X, labels = host[i]
    N, seed = inst[i][2], inst[i][3]
    tx, y = oracle.awgn(X, seed, s * N, N, math.sqrt(s2[i, s]))
    return oracle.gmi(oracle.llr_exact(X, labels, y, s2[i, s]), tx, labels)[0]


def test_every_class_of_the_mixed_sweep_against_oracle():
    """Each (M, D) class of the batched workload -- M in {16, 64, 256, 1024, 4096}, D in
    {2, 4, 8} -- at 2, 7 and 12 dB, against awgn -> llr_exact -> gmi of the FP64 oracle."""
    specs = [(M, D, 1500 + 97 * k) for k, (M, D) in enumerate(
        [(M, D) for M in (16, 64, 256, 1024, 4096) for D in (2, 4, 8)])]
    inst, host = make_instances(specs, seed=21)
    s2 = sigma2_grid(host, [2.0, 7.0, 12.0])
    for variant in (0, 3, 4):
        plan = md().SweepPlan(inst, s2, variant=variant)
        g = plan.run().cpu().numpy()
        n_fb, overflow = plan.stats()
        assert not overflow
        plan.close()
        for i in range(len(specs)):
            for s in range(3):
                gr = oracle_gmi(host, inst, s2, i, s)
                assert abs(g[i, s] - gr) <= 1e-4, (variant, specs[i], s, g[i, s], gr)


@pytest.mark.parametrize("variant", [0, 3])
def test_fp64_fallback_at_high_snr_against_oracle(variant):
    """At 20 and 24 dB the label-1 or label-0 subset of many symbols lies beyond the FP32
    range of the fast pass: those symbols take the FP64 fallback kernel, whose 2^-40
    fixed-point losses must still give the oracle's GMI.  Variant 0 runs two symbol blocks
    per wavefront (the received vectors parked in the staging rows for the fallback),
    variant 3 one block per wavefront (both lane halves draw, every other group, and a
    fallback symbol's received vector is drawn again)."""
    inst, host = make_instances([(2048, 8, 3000), (4096, 8, 2000), (1024, 4, 2500)], seed=33)
    s2 = sigma2_grid(host, [20.0, 24.0])
    plan = md().SweepPlan(inst, s2, variant=variant)
    g = plan.run().cpu().numpy()
    n_fb, overflow = plan.stats()
    assert n_fb > 0 and not overflow, (n_fb, overflow)
    for i in range(3):
        for s in range(2):
            gr = oracle_gmi(host, inst, s2, i, s)
            assert abs(g[i, s] - gr) <= 1e-4, (i, s, g[i, s], gr)
    # the graph replays give the same fallback count and the same GMIs
    g2 = plan.run().cpu().numpy()
    assert plan.stats() == (n_fb, False)
    assert np.array_equal(g, g2)
    plan.close()


def test_vector_kernel_fallback_at_high_snr_against_oracle():
    """The small-constellation vector kernel (shape 4) at 28 and 34 dB: symbols whose
    other-label subsets leave the FP32 range go to the FP64 fallback, and every GMI still
    matches the oracle."""
    inst, host = make_instances([(16, 2, 3000), (64, 4, 2000), (16, 8, 1500), (32, 3, 1200)], seed=44)
    s2 = sigma2_grid(host, [28.0, 34.0])
    plan = md().SweepPlan(inst, s2, variant=4)
    assert all(c[2] == 4 for c in plan.classes())
    g = plan.run().cpu().numpy()
    n_fb, overflow = plan.stats()
    assert n_fb > 0 and not overflow, (n_fb, overflow)
    for i in range(len(inst)):
        for s in range(2):
            gr = oracle_gmi(host, inst, s2, i, s)
            assert abs(g[i, s] - gr) <= 1e-4, (i, s, g[i, s], gr)
    plan.close()


def test_autotuner_per_class_shapes_and_cache():
    """With variant -1 every class gets its own measured launch shape; a second plan with
    the same classes takes them from the cache; variant 2 fixes one shape for all."""
    inst, host = make_instances(SPECS, seed=6)
    s2 = sigma2_grid(host, [4.0, 10.0])
    md().SweepPlan.tuning_clear()
    plan = md().SweepPlan(inst, s2, variant=-1)
    cls = plan.classes()
    assert len(cls) >= 3
    assert all(0 <= c[2] <= 4 for c in cls)
    # the vector kernel (shape 4) only for classes of at most 6 label bits
    assert all(c[2] != 4 or c[1] <= 6 for c in cls)
    assert sum(c[3] for c in cls) == plan.n_items
    ref = per_instance_gmi(inst, s2)
    np.testing.assert_allclose(plan.run().cpu().numpy(), ref, atol=1e-4, rtol=0)
    plan2 = md().SweepPlan(inst, s2, variant=-1)
    assert plan2.classes() == cls
    np.testing.assert_allclose(plan2.run().cpu().numpy(), ref, atol=1e-4, rtol=0)
    fixed = md().SweepPlan(inst, s2, variant=2)
    assert all(c[2] == 2 for c in fixed.classes())
    np.testing.assert_allclose(fixed.run().cpu().numpy(), ref, atol=1e-4, rtol=0)
    small = md().SweepPlan(inst, s2, variant=4)
    assert all(c[2] == (4 if c[1] <= 6 else 0) for c in small.classes())
    np.testing.assert_allclose(small.run().cpu().numpy(), ref, atol=1e-4, rtol=0)
    for p in (plan, plan2, fixed, small):
        p.close()
