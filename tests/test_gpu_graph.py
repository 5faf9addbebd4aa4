"""An apply recorded into a HIP graph (stream capture on the context stream)
replays to the eager result, bit for bit, on every replay, with eager work and
host synchronisations between replays; and contexts of different systems on
their own streams run concurrently without sharing state."""
import numpy as np
import pytest
import torch

from gen import trials_random
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _ctx(s, nb, prec, stream):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, stream=stream)


@pytest.mark.parametrize("cfg,prec", [("c1", "fp64"), ("p5", "fp64"), ("p5", "fp32")])
def test_graph_replay_matches_eager(systems, cfg, prec):
    s = systems(cfg)
    nb = s.cfg.nb
    st = torch.cuda.Stream()
    L = _ctx(s, nb, prec, st)
    inputs = [trials_random(s, nb, offset=2000 + 17 * k) for k in range(3)]
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = [torch.tensor(np.stack([x.real, x.imag], -1), dtype=dt, device="cuda").contiguous()
           for x in inputs]
    torch.cuda.synchronize()  # inputs made on the default stream, used on st
    say(f"graph capture cfg={cfg} prec={prec} nb={nb}")
    with torch.cuda.stream(st):
        eager = [L.apply(x).clone() for x in dev]
        a_in = dev[0].clone()
        a_out = torch.empty_like(a_in)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        L.apply(a_in, out=a_out)
    torch.cuda.synchronize()
    for rep in range(6):
        k = rep % 3
        # the replay runs on the context stream, after the copy and the clear
        # (torch's streams do not wait for the default stream, nor it for them)
        with torch.cuda.stream(st):
            a_in.copy_(dev[k])
            a_out.zero_()
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(a_out, eager[k]), f"replay {rep} differs from the eager apply"
        # eager work on the same context between replays
        with torch.cuda.stream(st):
            again = L.apply(dev[(k + 1) % 3])
        torch.cuda.synchronize()
        assert torch.equal(again, eager[(k + 1) % 3])
    say("  6 replays equal to the eager applies")
    del graph
    L.close()


def test_concurrent_contexts_on_own_streams(systems):
    cfgs = ["c1", "p1", "p2"]
    sys_ = [systems(c) for c in cfgs]
    streams = [torch.cuda.Stream() for _ in cfgs]
    ctxs = [_ctx(s, s.cfg.nb, "fp64", st) for s, st in zip(sys_, streams)]
    ins = [torch.tensor(np.stack([a.real, a.imag], -1), device="cuda").contiguous()
           for a in (trials_random(s, s.cfg.nb) for s in sys_)]
    torch.cuda.synchronize()
    say("concurrent contexts c1, p1, p2")
    ref = []
    for L, x, st in zip(ctxs, ins, streams):
        with torch.cuda.stream(st):
            ref.append(L.apply(x).clone())
        torch.cuda.synchronize()
    outs = [[torch.empty_like(x) for _ in range(3)] for x in ins]
    for rep in range(3):                      # interleaved launches, no host waits
        for i, (L, x, st) in enumerate(zip(ctxs, ins, streams)):
            with torch.cuda.stream(st):
                L.apply(x, out=outs[i][rep])
    torch.cuda.synchronize()
    for i in range(len(cfgs)):
        for rep in range(3):
            assert torch.equal(outs[i][rep], ref[i]), (cfgs[i], rep)
    for L in ctxs:
        L.close()
