"""GPU checks of the fused LLR + GMI pass (llr_exact_gmi), of the non-finite GMI status
(gmi_status) and of the failure paths under injected allocation failures
(alloc_fault_inject): MD_ENOMEM is returned, nothing leaks, the next call works."""
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


def setup(X, labels, snr, N, seed=5):
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, snr)
    tx, y = md().awgn_sample(Xd, seed, 0, N, math.sqrt(s2))
    return Xd, ld, s2, tx, y


@pytest.mark.parametrize("M,D,snr,N,prec", [(2048, 8, 4.0, 20011, "fp32"), (2048, 8, 14.0, 60000, "fp32"),
                                            (64, 4, 8.0, 30000, "fp32"), (256, 2, 25.0, 9000, "fp32"),
                                            (1024, 8, 9.0, 7000, "fp16"), (16, 2, 6.0, 5000, "fp32"),
                                            (4096, 4, 12.0, 5000, "bf16")])
def test_fused_gmi_matches_oracle_and_unfused(M, D, snr, N, prec):
    X, labels = synth.gaussian_constellation(M, D, M + D)
    if M == 64:
        X, labels = synth.product_4d_8psk()
    Xd, ld, s2, tx, y = setup(X, labels, snr, N)
    L, g, se = md().llr_exact_gmi(Xd, ld, y, tx, s2, prec=prec)
    L2 = md().llr_exact(Xd, ld, y, s2, prec=prec)
    assert torch.equal(L, L2)                    # the LLRs are llr_exact's
    g2, _, se2 = md().gmi_reduce(L2, tx, ld)
    assert abs(g.item() - g2.item()) <= 2e-5, (g.item(), g2.item())
    assert abs(se.item() - se2.item()) <= 1e-3 * se2.item() + 1e-9
    assert md().gmi_status() == 0
    if prec == "fp32":
        ref = oracle.llr_exact(X, labels, y.cpu().numpy(), s2)
        g_ref, _, _ = oracle.gmi(ref, tx.cpu().numpy().astype(np.uint32), labels)
        assert abs(g.item() - g_ref) <= 1e-4, (g.item(), g_ref)
    # deterministic
    _, g3, _ = md().llr_exact_gmi(Xd, ld, y, tx, s2, prec=prec)
    assert g3.item() == g.item()


def test_nonfinite_inputs_are_reported():
    X, labels = synth.gaussian_constellation(256, 4, 3)
    Xd, ld, s2, tx, y = setup(X, labels, 8.0, 4000)
    L = md().llr_exact(Xd, ld, y, s2)
    md().gmi_reduce(L, tx, ld)
    assert md().gmi_status() == 0
    L[17, 3] = float("nan")
    L[300, 0] = float("nan")
    g, _, _ = md().gmi_reduce(L, tx, ld)
    assert math.isnan(g.item())
    assert md().gmi_status() == 2
    lib = __import__("paper_2104_06311_amd._lib", fromlist=["lib"]).lib()
    import ctypes
    n = ctypes.c_int64()
    assert lib.gmi_status(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(n)) == -9
    assert n.value == 2 and b"non-finite" in lib.last_error()
    # a NaN received symbol through the fused path
    y2 = y.clone()
    y2[5, 1] = float("nan")
    _, g, _ = md().llr_exact_gmi(Xd, ld, y2, tx, s2)
    assert math.isnan(g.item()) and md().gmi_status() == 1
    # the next clean call clears the status
    md().llr_exact_gmi(Xd, ld, y, tx, s2)
    assert md().gmi_status() == 0


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def failure_round(Xd, ld, y, s2, ref, out, yl, lo, inst, sig, s, held0):
    """One pass over every injected allocation failure; each must give MD_ENOMEM and the
    call after it must work."""
    md().release_cache()
    with torch.cuda.stream(s):
        # after release_cache a stream's first call allocates its workspace, then its
        # stage counters
        md().alloc_fault_inject(1)           # the workspace succeeds, the counters fail
        with pytest.raises(md().MdemapError) as e:
            md().llr_exact(Xd, ld, y, s2, out=out)
        assert e.value.status == -5
        md().llr_exact(Xd, ld, y, s2, out=out)   # the injection fired once: this one works
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    md().release_cache()
    # a sweep plan that fails part-way through its allocations frees what it took
    for k in (0, 3, 6, 8):
        md().alloc_fault_inject(k)
        with pytest.raises(md().MdemapError) as e:
            md().SweepPlan(inst, sig, variant=0)
        assert e.value.status == -5, k
        assert md().alloc_stats() == held0, k
    md().alloc_fault_inject(-1)
    # a network whose parameter allocation fails, and one whose inference image does
    md().alloc_fault_inject(0)
    with pytest.raises(md().MdemapError) as e:
        md().MLP(8, 64, 10, seed=1)
    assert e.value.status == -5
    assert md().alloc_stats() == held0
    net = md().MLP(8, 64, 10, seed=1)
    held = md().alloc_stats()
    md().alloc_fault_inject(0)
    with pytest.raises(md().MdemapError) as e:
        md().llr_learned(net, yl, out=lo)
    assert e.value.status == -5
    assert md().alloc_stats() == held
    md().llr_learned(net, yl, out=lo)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(lo).all().item())
    net.close()
    md().alloc_fault_inject(-1)
    md().release_cache()


def test_injected_allocation_failures_leak_nothing():
    """Every failure path returns MD_ENOMEM and frees what it had taken: the library's own
    count of live device allocations is back at zero after each failed creation and after
    release_cache, over six rounds; and the device's free memory does not shrink round
    after round (a plan leaking its 40 MiB fallback queue would show five times over)."""
    X, labels = synth.gaussian_constellation(1024, 8, 9)
    Xd, ld, s2, tx, y = setup(X, labels, 9.0, 50_000)
    ref = md().llr_exact(Xd, ld, y, s2)
    out = torch.empty_like(ref)
    yl = torch.randn((1000, 8), device="cuda")
    lo = torch.empty((1000, 10), device="cuda")
    g = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    inst = [(Xd, ld, 20000, 3)]
    sig = np.array([[s2, s2 / 2]])
    s = torch.cuda.Stream()
    md().release_cache()
    held0 = md().alloc_stats()          # handles of earlier work still alive, if any
    failure_round(Xd, ld, y, s2, ref, out, yl, lo, inst, sig, s, held0)
    assert md().alloc_stats() == held0
    torch.cuda.empty_cache()
    base = free_bytes()
    for _ in range(5):
        failure_round(Xd, ld, y, s2, ref, out, yl, lo, inst, sig, s, held0)
        assert md().alloc_stats() == held0
    torch.cuda.empty_cache()
    after = free_bytes()
    assert after >= base - (64 << 20), (base, after)
    plan = md().SweepPlan(inst, sig, variant=0)   # and the same calls work afterwards
    assert md().alloc_stats()[1] > held0[1]
    plan.run(out=g)
    assert np.all(np.isfinite(g.cpu().numpy()))
    plan.close()
    assert md().alloc_stats() == held0
