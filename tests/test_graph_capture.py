"""gf_scan_noalloc recorded into a HIP graph.  It allocates nothing and
enqueues only kernels (node tables, subtraction sums, the scan; no memset),
so a caller can capture it: every replay, with eager work and
synchronisations between the replays, gives the eager call's bits."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1205_0752_amd as gf  # noqa: E402
from paper_1205_0752_amd.workloads import Grid, Params, Quadrature  # noqa: E402

pytestmark = pytest.mark.gpu


def test_noalloc_scan_replays_from_a_graph_like_the_eager_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()
    p, q, grid = (Params(1 + 0.5j, 1 - 0.5j, 1.0, 1e6), Quadrature(64, 33, 16),
                  Grid(45, 37, -12.0, 6.0, -6.0, 6.0))
    p2, q2, grid2 = Params(1.0, 0.25, 2.0, 1e4), Quadrature(48, 24, 8), Grid(19, 11, -7.0, 5.0, -3.0, 4.5)
    s = torch.cuda.Stream()
    out = gf.empty_result(grid)
    with torch.cuda.stream(s):
        gf.scan_noalloc(p, grid, q, out)  # eager; also looks up the static buffer
    s.synchronize()
    ref = out.cpu().numpy().view(np.float64).copy()
    graph = torch.cuda.CUDAGraph()
    out.fill_(complex(float("nan"), 0.0))
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        gf.scan_noalloc(p, grid, q, out)
    for _ in range(3):
        out.fill_(complex(float("nan"), 0.0))
        # eager work between the replays: another scan that refills the same
        # static buffer with other node tables
        other = gf.empty_result(grid2)
        gf.scan_noalloc(p2, grid2, q2, other)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.float64)
        assert np.array_equal(got, ref, equal_nan=True)
        assert np.isfinite(other.cpu().numpy()).any()
