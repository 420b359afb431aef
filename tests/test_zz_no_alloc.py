"""The allocation-free entry point gks_run1d_noalloc against the handle path
(gks_init_device / gks_step / gks_state) on the GPU: same kernels, so the
results must be bit-identical.  Two calls in a row, the second with a
smaller problem (the static scratch array is re-initialised by every call),
then a run split over two calls that continue in time."""
import numpy as np
import pytest

from paper_1901_00261_amd import workloads as wl

pytestmark = pytest.mark.gpu


def gks():
    from paper_1901_00261_amd import gks as g
    return g


def handle_run(p, steps, precision):
    g = gks()
    S = g.Solver(p, precision)
    S.step(steps, raise_on_error=False)
    W, Wx, _, t, n = S.state(0)
    st = S.status(0)
    S.close()
    return W, Wx, t, n, st


def noalloc_run(p, steps, precision, t0=0.0, arrays=None):
    import torch
    g = gks()
    dev = torch.device("cuda:0")
    if arrays is None:
        arrays = (torch.from_numpy(np.ascontiguousarray(p.W)).to(dev), torch.from_numpy(np.ascontiguousarray(p.Wx)).to(dev))
    W, Wx = arrays
    stream = torch.cuda.current_stream().cuda_stream
    t, n, st = g.run1d_noalloc(p, W.data_ptr(), Wx.data_ptr(), steps, t0=t0, precision=precision, stream=stream)
    torch.cuda.synchronize()
    return W.cpu().numpy(), Wx.cpu().numpy(), t, n, st, arrays


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_handle_path(precision):
    big = wl.riemann_set_1d(1, n=900)[0]
    small = wl.sine_wave_1d(40, order=6, recon=1, t_end=2.0)
    for p, steps in ((big, 60), (small, 25)):
        want = handle_run(p, steps, precision)
        got = noalloc_run(p, steps, precision)
        print(p.name, p.nx, "steps", got[3], "t", got[2], "status", got[4], flush=True)
        assert got[3] == want[3] == steps and got[2] == want[2] and got[4] == want[4] == 0
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_noalloc_split_run_continues_in_time_and_stops_at_t_end():
    p = wl.riemann_1d(300, *wl.SOD, t_end=0.05)
    want = handle_run(p, 100000, 0)
    assert want[4] == 1
    W1, Wx1, t1, n1, st1, arrays = noalloc_run(p, 40, 0)
    assert n1 == 40 and st1 == 0
    # five more steps than needed: the finished problem skips them
    W2, Wx2, t2, n2, st2, _ = noalloc_run(p, want[3] - 40 + 5, 0, t0=t1, arrays=arrays)
    assert st2 == 1 and t2 == want[2] == 0.05 and n1 + n2 == want[3]
    assert np.array_equal(W2, want[0]) and np.array_equal(Wx2, want[1])


def test_noalloc_rejects_oversized_and_2d_problems():
    """Host-side validation before anything is enqueued (real device
    buffers are passed all the same)."""
    import torch
    g = gks()
    big = wl.riemann_1d(40000, *wl.SOD)
    W = torch.zeros((40000, 4), dtype=torch.float64, device="cuda:0")
    with pytest.raises(g.GksError) as e:
        g.run1d_noalloc(big, W.data_ptr(), W.data_ptr(), 1)
    assert e.value.code == g.GKS_EINVAL and "scratch limit" in str(e.value)
    p2 = wl.isentropic_vortex_2d(8)
    with pytest.raises(g.GksError) as e:
        g.run1d_noalloc(p2, W.data_ptr(), W.data_ptr(), 1)
    assert e.value.code == g.GKS_EINVAL
    torch.cuda.synchronize()
