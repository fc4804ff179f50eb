"""The accuracy-sweep harness on a small grid: the batched estimator's fields
match the FP64 oracle's, and so does their Psi score (Psi moves by at most
the largest field difference, since it averages absolute magnitudes)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import metrics as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ofv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_25924_amd as m
    m.load()
    return m


def test_small_rankine_sweep_matches_oracle(ofv):
    say("mini sweep")
    S = 96
    c = (S - 1) / 2.0
    imgs = [(3.0, 12.0), (4.0, 20.0)]          # (max displacement, core radius)
    vort = [synth.Rankine(c, c, R, D) for D, R in imgs]
    pairs = [synth.make_pair(S, S, v, fwhm=0.75 * synth.FWHM_PER_SIGMA * 2.0, ppp=10 / 256.0, seed=70 + i,
                             bit_depth=8, noise=0.0) for i, v in enumerate(vort)]
    f0 = [torch.from_numpy(p.frame0).cuda() for p in pairs]
    f1 = [torch.from_numpy(p.frame1).cuda() for p in pairs]
    h = ofv.Handle(S, S, len(imgs))
    for kr, psl, it, nr in [(2, 2, 2, 1), (4, 2, 3, 2)]:
        prm = {"num_levels": psl + 1, "kernel_radius": kr, "iterations": it, "norm_radius": nr}
        got = ofv.compute_flow_batch(f0, f1, prm, bit_depth=8, handle=h)
        for i, (p, v) in enumerate(zip(pairs, vort)):
            ref = oracle.compute_flow(p.frame0, p.frame1, prm, bit_depth0=8)
            d = torch.max(torch.abs(got[i].cpu().double() - ref)).item()
            g_psi = M.psi(got[i][None].double(), v).item()
            o_psi = M.psi(ref[None].cuda(), v).item()
            say(f"  KR {kr} PSL {psl} IT {it} NR {nr} image {i}: max |dV| {d:.2e}, psi {g_psi:.4f} / {o_psi:.4f}")
            assert d <= 1e-3
            assert abs(g_psi - o_psi) <= d + 1e-9
    h.close()
