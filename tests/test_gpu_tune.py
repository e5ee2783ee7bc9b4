"""GPU test of the sweep autotuner (rpca_autotune) and of its use.

The tuner times rpca_objgrad on a probe instance for every candidate
decomposition of every (k, n) bucket and keeps the fastest.  Checked here:
it runs on the device and leaves every entry at one of its candidates;
contexts created afterwards take their decomposition from the table
(rpca_sweep_layout) and stay at oracle parity (FP32 bar, 1e-5) under a
non-default entry; batches scale their instances' wave shares by the entry.
The table is process-wide, so the test restores it before it ends.
"""
import numpy as np
import pytest
import torch

from oracle import objective as ob
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32, rel

pytestmark = pytest.mark.gpu

K_REP = [8, 16, 24, 32]
N_REP = [64, 128, 256, 512, 1024]
WAVE_CAND = {1024, 2048, 4096}
DIV_CAND = {1, 2}


@pytest.fixture
def saved_table():
    saved = {(k, n): R.rpca_tune_get(k, n)[1:] for k in K_REP for n in N_REP}
    yield saved
    for (k, n), (w, d) in saved.items():
        assert R.rpca_tune_set(k, n, w, d) == R.RPCA_OK


def test_autotune_runs_and_contexts_use_the_table(saved_table):
    device()
    rc = R.rpca_autotune(4096, 3, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == R.RPCA_OK
    tuned = {(k, n): R.rpca_tune_get(k, n)[1:] for k in K_REP for n in N_REP}
    changed = sum(tuned[key] != saved_table[key] for key in tuned)
    print(f"[autotune m_probe=4096] {changed} of {len(tuned)} entries changed: "
          + " ".join(f"k{k}n{n}={w}/{d}" for (k, n), (w, d) in sorted(tuned.items())), flush=True)
    for w, d in tuned.values():
        assert w in WAVE_CAND and d in DIV_CAND

    # a context made after a table change takes the entry's decomposition
    p = synth.gaussian_rpca(m=20000, n=200, r=5, k=10, seed=77)
    U0, V0 = synth.random_factors(p.m, p.n, p.k, 78, scale=0.4)
    dev = device()
    Xcm = T.to_device_X(p.X, dev)
    Ud, Vd = T.to_device_factor(U0, dev), T.to_device_factor(V0, dev)
    fr, gUr, gVr = ob.objgrad(f32(U0), f32(V0), f32(p.X), p.lam_s, p.lam_l)
    layouts = {}
    for w, d in [(1024, 1), (4096, 2)]:
        assert R.rpca_tune_set(p.k, p.n, w, d) == R.RPCA_OK
        ctx = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l)
        rc, lay = R.rpca_sweep_layout(ctx.ctx)
        assert rc == R.RPCA_OK
        layouts[(w, d)] = lay
        f, gU, gV = ctx.objgrad(Xcm, Ud, Vd)
        torch.cuda.synchronize()
        ef = abs(f.item() - fr) / abs(fr)
        eu, ev = rel(gU.cpu().numpy(), gUr), rel(gV.cpu().numpy(), gVr)
        print(f"[tuned entry {w}/{d}] layout (rows, strips/wave, chunk, chunks) = {lay}; "
              f"f rel {ef:.2e} gU rel {eu:.2e} gV rel {ev:.2e}", flush=True)
        assert ef <= 1e-5 and eu <= 1e-5 and ev <= 1e-5
        ctx.close()
    a, b = layouts[(1024, 1)], layouts[(4096, 2)]
    assert b[0] * b[3] > a[0] * a[3]     # more workgroups for the larger wave target
    assert b[2] < a[2] and b[3] > a[3]   # the chunk divisor halves the widest chunk

    # a batch scales each instance's wave share by its bucket's entry
    shapes = [(8192, 200, 10), (4096, 100, 8)]
    waves = {}
    for w in (1024, 4096):
        for (m, n, k) in shapes:
            assert R.rpca_tune_set(k, n, w, 1) == R.RPCA_OK
        B = T.Batch(shapes, [0.05, 0.05], [1.0, 1.0])
        waves[w] = [B.instance_waves(i) for i in range(len(shapes))]
        B.close()
    print(f"[batch wave shares] table 1024: {waves[1024]}  table 4096: {waves[4096]}", flush=True)
    assert all(hi >= lo for hi, lo in zip(waves[4096], waves[1024]))
    assert any(hi > lo for hi, lo in zip(waves[4096], waves[1024]))
