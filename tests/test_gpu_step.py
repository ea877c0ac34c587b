"""GPU test of the benchmark's E-REMD step as a runtime: the Monte Carlo branch
on a second stream beside the force passes, double-buffered charges, and the
two-parity hipGraph replays give exactly the states, charges, ladder and
counters of the plain single-stream eager sequence."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _run(overlap, use_graph, n_steps):
    import bench
    w = bench.Workload("fp32", n_steps + 2, bench.DEFAULT_ORDER, None, overlap)
    k = 0
    graphs = None
    if use_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(2):
                w.step(k % 2)
                k += 1
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs = []
        for parity in (0, 1):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                w.step(parity)
            graphs.append(gr)
    snaps = []
    while k < n_steps:
        if graphs is not None:
            graphs[k % 2].replay()
        else:
            w.step(k % 2)
        k += 1
        torch.cuda.synchronize()
        q = (w.atoms if k % 2 == 0 else w.atoms_b).q
        snaps.append({"q": q.cpu().numpy().copy(), "state": w.cur.cpu().numpy().copy(),
                      "E_rep": w.E_rep.cpu().numpy().copy(),
                      "rep": w.rep_of_rung.cpu().numpy().copy(),
                      "counters": w.counters.cpu().numpy().copy()})
    return snaps


def test_overlapped_graph_step_equals_serial_eager_step():
    n = 12
    ref = _run(overlap=False, use_graph=False, n_steps=n)
    got = _run(overlap=True, use_graph=True, n_steps=n)
    # the graph run's first two steps are its eager capture warm-up
    assert len(got) == n - 2 and len(ref) == n
    for a, b in zip(got, ref[2:]):
        for key in a:
            assert np.array_equal(a[key], b[key]), key
    # the Monte Carlo chain moved: some attempts were accepted
    assert ref[-1]["counters"][:, 1].sum() > 0


def test_two_step_graph_equals_serial_eager_steps():
    # the benchmark's replay loop: one graph holding an even and an odd step
    # back to back; after every replay the state equals the eager sequence's
    import bench
    n = 12
    ref = _run(overlap=False, use_graph=False, n_steps=n)
    w = bench.Workload("fp32", n + 2, bench.DEFAULT_ORDER, None, True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        w.step(0)
        w.step(1)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    pair = torch.cuda.CUDAGraph()
    with torch.cuda.graph(pair):
        w.step(0)
        w.step(1)
    k = 2
    while k + 2 <= n:
        pair.replay()
        k += 2
        torch.cuda.synchronize()
        b = ref[k - 1]
        assert np.array_equal(w.atoms.q.cpu().numpy(), b["q"])
        assert np.array_equal(w.cur.cpu().numpy(), b["state"])
        assert np.array_equal(w.E_rep.cpu().numpy(), b["E_rep"])
        assert np.array_equal(w.rep_of_rung.cpu().numpy(), b["rep"])
        assert np.array_equal(w.counters.cpu().numpy(), b["counters"])
