"""Time-resolved streaming: each pushed frame is normalised and reduced once
and paired with the next one.  Every produced field must equal the pair
computation of the same two frames bit for bit (same kernels on the same
planes), and one of them is checked against the FP64 oracle directly."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

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


def _sequence(n_frames, h=200, w=240, step=(2, -1), seed=31):
    """Crops of one particle texture moving by an integer step per frame, 12-bit with noise."""
    m = 4 + n_frames * max(abs(step[0]), abs(step[1]))
    tex = synth.make_texture(h, w, fwhm=2.5, ppp=0.1, seed=seed, margin=m)
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n_frames):
        y0, x0 = m - t * step[1], m - t * step[0]
        f = tex[y0:y0 + h, x0:x0 + w] * 3000.0 + rng.normal(0, 20.0, (h, w))
        out.append(np.clip(np.rint(f), 0, 4095).astype(np.uint16))
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_pushed_fields_equal_pair_calls(ofv, storage):
    say("stream", storage)
    frames = [torch.from_numpy(f).cuda() for f in _sequence(5)]
    prm = {"num_levels": 3, "kernel_radius": 4, "iterations": 3, "norm_radius": 1, "storage": storage}
    hs = ofv.Handle(240, 200, 1)
    hp = ofv.Handle(240, 200, 1)
    assert hs.stream_push(frames[0], prm, bit_depth=12) is None
    prev = None
    for t in range(1, 5):
        init = prev.clone() if (prev is not None and t % 2 == 0) else None   # warm start on even steps
        got = hs.stream_push(frames[t], prm, flow_init=init, bit_depth=12)
        ref = ofv.compute_flow(frames[t - 1], frames[t], prm, flow_init=init, bit_depth=12, handle=hp)
        torch.cuda.synchronize()
        assert got is not None and torch.equal(got, ref), t
        prev = got
    hs.close()
    hp.close()


def test_pushed_field_matches_oracle(ofv):
    say("stream vs oracle")
    seq = _sequence(2, 160, 176)
    prm = {"num_levels": 3, "kernel_radius": 4, "iterations": 3, "norm_radius": 1}
    h = ofv.Handle(176, 160, 1)
    h.stream_push(torch.from_numpy(seq[0]).cuda(), prm, bit_depth=12)
    got = h.stream_push(torch.from_numpy(seq[1]).cuda(), prm, bit_depth=12)
    ref = oracle.compute_flow(seq[0], seq[1], prm, bit_depth0=12)
    err = torch.max(torch.abs(got.cpu().double() - ref)).item()
    say("  max |dV| =", err)
    assert err <= 1e-3
    h.close()


def test_other_calls_and_parameter_changes_restart_the_stream(ofv):
    say("stream restarts")
    frames = [torch.from_numpy(f).cuda() for f in _sequence(4)]
    prm = {"num_levels": 3, "kernel_radius": 4, "iterations": 3, "norm_radius": 1}
    h = ofv.Handle(240, 200, 1)
    assert h.stream_push(frames[0], prm, bit_depth=12) is None
    assert h.stream_push(frames[1], dict(prm, kernel_radius=3, iterations=2), bit_depth=12) is not None
    with pytest.raises(ofv.OfvError):
        h.stream_push(frames[2], dict(prm, num_levels=2), bit_depth=12)
    with pytest.raises(ofv.OfvError):
        h.stream_push(frames[2][:100], prm, bit_depth=12)
    assert h.stream_push(frames[2], prm, bit_depth=12) is not None   # a refused push keeps the stream
    ofv.compute_flow(frames[0], frames[1], prm, bit_depth=12, handle=h)  # reuses the workspace
    assert h.stream_push(frames[3], prm, bit_depth=12) is None
    h.stream_reset()
    assert h.stream_push(frames[0], dict(prm, num_levels=2), bit_depth=12) is None
    assert h.stream_push(frames[1], dict(prm, num_levels=2), bit_depth=12) is not None
    h.close()


def test_captured_pushes_alternate(ofv):
    """Two captured pushes (new frame into slab 1, then into slab 0), replayed
    alternately over new frames copied into their input buffers."""
    say("stream graph")
    seq = [torch.from_numpy(f).cuda() for f in _sequence(7)]
    prm = {"num_levels": 3, "kernel_radius": 4, "iterations": 3, "norm_radius": 1}
    h = ofv.Handle(240, 200, 1)
    hp = ofv.Handle(240, 200, 1)
    bufs = [torch.empty_like(seq[0]) for _ in range(2)]
    outs = [torch.empty((2, 200, 240), dtype=torch.float32, device="cuda") for _ in range(2)]
    bufs[0].copy_(seq[0])
    h.stream_push(bufs[0], prm, bit_depth=12)          # retained frame in slab 0
    graphs = []
    for k in range(2):                                 # push into slab 1, then slab 0
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            h.stream_push(bufs[(k + 1) % 2], prm, bit_depth=12, out=outs[k])
        graphs.append(g)
    h.bind_stream()
    # the captures enqueued nothing: rebuild the retained frame, then replay
    h.stream_reset()
    bufs[0].copy_(seq[0])
    h.stream_push(bufs[0], prm, bit_depth=12)
    for t in range(1, 7):
        k = (t - 1) % 2
        bufs[(k + 1) % 2].copy_(seq[t])
        graphs[k].replay()
        ref = ofv.compute_flow(seq[t - 1], seq[t], prm, bit_depth=12, handle=hp)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], ref), t
    h.close()
    hp.close()
