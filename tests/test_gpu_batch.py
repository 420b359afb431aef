"""Batched 1-D path: launch configurations, graph replay, autotuner (GPU).

Every launch configuration (tile of 64/128/256 threads, persistent grid of
GMUL workgroups per CU or one workgroup per work item) runs the same
per-face and per-cell arithmetic, so all must agree bit for bit; the batch
must also match the oracle problem by problem.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1901_00261_amd import workloads as wl

pytestmark = pytest.mark.gpu


def gks():
    from paper_1901_00261_amd import gks as g
    return g


def run(probs, steps=None, tune=None, graph=None, precision=0, split=None, phases=None):
    g = gks()
    old = {k: os.environ.get(k) for k in ("GKS_TUNE", "GKS_GRAPH", "GKS_SPLIT", "GKS_PHASES")}
    try:
        for k, v in (("GKS_TUNE", tune), ("GKS_GRAPH", graph), ("GKS_SPLIT", split), ("GKS_PHASES", phases)):
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        S = g.Solver(probs, precision)
        if steps is None:
            while S.step(1000) > 0:
                pass
        else:
            S.step(steps)
        cfg = S.launch_config()
        out = [S.state(p) for p in range(len(probs))]
        S.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return out, cfg


@pytest.fixture(scope="module")
def batch():
    return wl.batch_1d(count=12, seed=7, nmin=40, nmax=700, t_end=0.05)


@pytest.mark.parametrize("tune", ["64:0", "64:1", "128:2", "256:0", "256:4"])
def test_launch_modes_bit_identical(batch, tune):
    # the reference runs the single-lane kernel throughout; with its 36 work
    # items the compared run switches to the lane-pair kernel after its
    # first call
    ref, _ = run(batch, tune="128:0", graph="0", split="0")
    got, cfg = run(batch, tune=tune)
    assert cfg.startswith("forced")
    for a, b in zip(ref, got):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4] and a[3] == b[3]


@pytest.mark.parametrize("tune", ["64:1", "256:0"])
def test_launch_modes_bit_identical_mixed(batch, tune):
    ref, _ = run(batch, tune="128:0", graph="0", precision=1, split="0")
    got, _ = run(batch, tune=tune, precision=1)
    for a, b in zip(ref, got):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4]


@pytest.mark.parametrize("precision", [0, 1])
def test_lane_pair_steps_bit_identical(batch, precision):
    """The lane-pair kernel (two lanes share a face: one WENO-Z side and one
    non-equilibrium state each, exchanged by DPP moves) reproduces the
    single-lane kernel bit for bit: on for the whole run against off."""
    ref, cfg0 = run(batch, split="0", precision=precision)
    got, cfg = run(batch, split="2", precision=precision)
    assert "lane-pair steps off" in cfg0 and "lane-pair steps on" in cfg
    for a, b in zip(ref, got):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4] and a[3] == b[3]


@pytest.mark.parametrize("precision", [0, 1])
def test_two_kernel_steps_bit_identical(batch, precision):
    """Two-kernel steps (face kernel, the reconstructed faces through HBM,
    then the point-and-cell kernel) reproduce the fused kernel bit for bit:
    on for the whole run against off."""
    ref, cfg0 = run(batch, split="0", phases="0", precision=precision)
    got, cfg = run(batch, split="0", phases="2", precision=precision)
    assert "two-kernel steps off" in cfg0 and "two-kernel steps on" in cfg
    for a, b in zip(ref, got):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4] and a[3] == b[3]


def test_step_form_switches_during_a_run():
    """The 256-problem uneven batch: two-kernel steps while its work items
    fill the CUs, fused steps below that, lane-pair steps once the items are
    at most half the CUs; every problem ends bit-identical to a run in the
    fused form throughout."""
    g = gks()
    probs = wl.batch_1d(t_end=0.02)

    def go(split, phases):
        old = {k: os.environ.get(k) for k in ("GKS_SPLIT", "GKS_PHASES")}
        os.environ["GKS_SPLIT"] = split
        os.environ["GKS_PHASES"] = phases
        try:
            S = g.Solver(probs)
            # three problems of this batch meet a non-physical state in
            # their first steps and stop; the others run on
            S.step(1, raise_on_error=False)
            S.step(1, raise_on_error=False)
            cfg_first = S.launch_config()
            # calls of 100 steps, so that the switches (decided at each call
            # from the work items left after the previous one) come while
            # the largest problems still run
            while S.step(100, raise_on_error=False) != 0:
                pass
            out = [S.state(p) + (S.status(p),) for p in range(len(probs))]
            cfg = S.launch_config()
            S.close()
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        return out, cfg_first, cfg

    ref, _, cfg0 = go("0", "0")
    got, cfg1, cfg = go("1", "1")
    assert "lane-pair steps off" in cfg0 and "two-kernel steps off" in cfg0
    assert "two-kernel steps on" in cfg1
    assert "lane-pair steps on" in cfg and "two-kernel steps off" in cfg
    assert sum(r[5] == g.GKS_ENONPHYS for r in ref) == 3
    for a, b in zip(ref, got):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4] and a[3] == b[3]
        assert a[5] == b[5]


def test_bad_tune_string_is_rejected(batch):
    g = gks()
    os.environ["GKS_TUNE"] = "persistent"
    try:
        S = g.Solver(batch[:2])
        with pytest.raises(g.GksError) as e:
            S.step(1)
        assert e.value.code == g.GKS_EINVAL and "GKS_TUNE" in str(e.value)
        S.close()
    finally:
        os.environ.pop("GKS_TUNE")


def test_batch_matches_oracle(batch):
    got, cfg = run(batch)
    print("autotuned:", cfg)
    for p, g in zip(batch, got):
        want = oracle.run(1, p.W, p.Wx, **p.oracle_kwargs())
        err = np.abs(g[0] - want[0]).max() / np.abs(want[0]).max()
        assert g[4] == want[4] and err < 1e-10, (p.nx, err)


@pytest.fixture(scope="module")
def long_smooth():
    """Two smooth problems large enough for many work items; the oracle after 6 steps."""
    probs = [wl.sine_wave_1d(40000, order=8, recon=1), wl.sine_wave_1d(30000, order=6, recon=1)]
    want = [oracle.run(1, p.W, p.Wx, **{**p.oracle_kwargs(), "max_steps": 6}) for p in probs]
    return probs, want


@pytest.mark.parametrize("tune", ["256:1", "64:1"])
def test_items_over_several_rounds_match_oracle(long_smooth, tune):
    """More work items than workgroups (one workgroup per CU: 275 items of 255
    cells, or 1 112 items of 63 cells), so items start after neighbouring items
    of the same problem have finished.  Such an item must still read its
    neighbours' edge cells at the half step (reading them after the update
    would shift W by about dt |W_t| ~ 1e-5): every cell of both problems
    matches the oracle.  Values: relative L-inf <= 1e-11.  Gradients are
    differences of neighbouring face values divided by dx, so rounding
    differences of the face values (a few hundred eps |W| between the two
    implementations) grow by 1/dx: the bar is 256 eps max|W| / dx on top of
    1e-11 max|W_x| (4e-9 absolute at 40 000 cells)."""
    probs, want = long_smooth
    got, cfg = run(probs, steps=6, tune=tune)
    assert cfg.startswith("forced")
    eps = np.finfo(np.float64).eps
    for p, g, w in zip(probs, got, want):
        assert g[4] == w[4] == 6
        err = np.abs(g[0] - w[0]).max() / np.abs(w[0]).max()
        assert err <= 1e-11, (p.nx, err)
        dx = (p.xhi - p.xlo) / p.nx
        bar = 1e-11 * np.abs(w[1]).max() + 256 * eps * np.abs(w[0]).max() / dx
        errx = np.abs(g[1] - w[1]).max()
        print(f"N={p.nx} {tune}: W {err:.2e}, W_x {errx:.2e} (bar {bar:.2e})")
        assert errx <= bar, (p.nx, errx, bar)


def test_graph_replays_match_eager_with_host_reads(batch):
    g = gks()
    os.environ["GKS_TUNE"] = "128:2"
    try:
        os.environ["GKS_GRAPH"] = "1"
        A = g.Solver(batch)
        os.environ["GKS_GRAPH"] = "0"
        B = g.Solver(batch)
    finally:
        os.environ.pop("GKS_GRAPH", None)
        os.environ.pop("GKS_TUNE", None)
    for rep in range(6):
        n = 3 if rep % 2 == 0 else 11  # 11: one eight-step replay and three one-step replays
        A.step(n)
        B.step(n)
        for p in (0, 5, 11):  # host reads between replays
            a, b = A.state(p), B.state(p)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4], (rep, p)
    A.close()
    B.close()


def test_tune_cache_round_trip(tmp_path, batch):
    cache = tmp_path / "tune.txt"
    os.environ["GKS_TUNE_CACHE"] = str(cache)
    try:
        _, cfg1 = run(batch[:4], steps=2)
        assert cfg1.startswith("tuned") and cache.exists()
        _, cfg2 = run(batch[:4], steps=2)
        assert cfg2.startswith("cache")
    finally:
        os.environ.pop("GKS_TUNE_CACHE", None)


def test_2d_graph_matches_eager():
    p = wl.isentropic_vortex_2d(24, ny=20, mu=1e-3, acoustic_amp=1e-2)
    g = gks()
    os.environ["GKS_GRAPH"] = "0"
    try:
        B = g.Solver(p)
    finally:
        os.environ.pop("GKS_GRAPH")
    A = g.Solver(p)
    for rep in range(3):
        n = 2 if rep != 1 else 9  # 9: one eight-step replay and one one-step replay
        A.step(n)
        B.step(n)
        a, b = A.state(0), B.state(0)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    A.close()
    B.close()
