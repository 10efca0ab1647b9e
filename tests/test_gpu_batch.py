"""Batched Reynolds sweeps: one persistent launch per stage solves every cavity
(grid barriers between sweep rounds, per-cavity stopping decisions on the
device), optionally with the whole step captured in a hipGraph.

A persistent round is the same arithmetic as one launch of the per-cavity
path, so with the same sweeps per launch, check spacing and relaxation the
batched results are bitwise those of each cavity run on its own.
"""
import numpy as np
import pytest

from oracle.cavity_oracle import CavityOracle

pytestmark = pytest.mark.gpu

# a compiled per-launch FP64 sweep kernel for each number of sweeps per launch
SOLO_TILES = {1: (32, 32, 256), 2: (64, 64, 1024), 3: (64, 64, 1024), 4: (64, 64, 512),
              5: (84, 54, 1024)}
SMALL4 = [(5000.0, 130), (10000.0, 257), (15000.0, 384), (20000.0, 512)]
SWEEP6 = [(5000.0, 256), (10000.0, 512), (15000.0, 768), (20000.0, 1024), (25000.0, 1024),
          (30000.0, 1024)]


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


def _solo(cm, n, re, precision, s, check_every, inner):
    c = cm.Cavity(cm.Params(n=n, re=re, precision=precision))
    t = c.tuning()
    c.set_tuning(tile_x=64, tile_y=64, sweeps_per_launch=s, threads=1024,
                 tile_x32=64, tile_y32=64, sweeps_per_launch32=s, threads32=1024,
                 check_every=check_every, inner_sweeps=inner, xcd_bands=0,
                 sor_omega=t["sor_omega"])
    return c


@pytest.mark.parametrize("mode", ["persistent", "graph"])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_bitwise_equals_solo_runs(cm, mode, precision):
    """Every step (every graph replay, with host work in between) is compared."""
    members = [(5000.0, 130), (10000.0, 200), (15000.0, 257)]
    steps, s, check_every, inner = 4, 2, 8, 256
    print(f"[batch {mode} precision={precision}] {members}", flush=True)
    c = cm.Cavity([cm.Params(n=n, re=re, precision=precision) for re, n in members])
    c.set_exec(cm.CAVITY_EXEC_PERSISTENT if mode == "persistent" else cm.CAVITY_EXEC_GRAPH)
    c.set_tuning(-1, tile_x=64, tile_y=64, sweeps_per_launch=s, threads=512,
                 tile_x32=64, tile_y32=64, sweeps_per_launch32=s, threads32=1024,
                 check_every=check_every, inner_sweeps=inner)
    solos = [_solo(cm, n, re, precision, s, check_every, inner) for re, n in members]
    for step in range(steps):
        stats = c.step(1)
        for k, solo in enumerate(solos):
            st = solo.step(1)[0]
            p, w, _, _ = solo.fields()
            gp, gw, _, _ = c.fields(k)
            assert np.array_equal(gp, p), (step, k)
            assert np.array_equal(gw, w), (step, k)
            assert stats[k]["sweeps_last_step"] == st["sweeps_last_step"], (step, k)
            assert stats[k]["status"] == 0
    c.close()
    for solo in solos:
        solo.close()


def test_reynolds_sweep_six_cavities_graph(cm):
    """The six-cavity Reynolds sweep (256^2 ... 1024^2) in graph mode, every
    member against the oracle at 1e-11.

    A few steps from rest psi is still small (max |psi| of order 1e-3), and a
    solve that stops as soon as its residual is below the tolerance t leaves
    an error up to ||A^-1|| t = 0.074 t in psi: relative to max |psi| that is
    above 1e-11 for t = 1e-10 (the error of the extrapolated starts often
    sits near it, since their solves stop at the first check below t).  The
    run solves to 1e-11, where the bar checks the execution mode rather than
    the tolerance."""
    members = SWEEP6
    steps = 3
    print("[re sweep] six cavities", flush=True)
    c = cm.Cavity([cm.Params(n=n, re=re, poisson_tol=1e-11) for re, n in members])
    # cavities this large default to a stream each; the graph is still there
    assert c.exec_mode() == cm.CAVITY_EXEC_STREAM
    c.set_exec(cm.CAVITY_EXEC_GRAPH)
    stats = c.step(steps)
    fields = [c.fields(k) for k in range(len(members))]
    c.close()
    for k, (re, n) in enumerate(members):
        psi, omega = fields[k][0], fields[k][1]
        assert stats[k]["status"] == 0 and stats[k]["step"] == steps
        assert np.all(psi[0, :] == 0) and np.all(psi[-1, :] == 0)
        assert np.all(psi[:, 0] == 0) and np.all(psi[:, -1] == 0)
        assert np.all(np.isfinite(omega))
    # every member against the oracle
    for k, (re, n) in enumerate(members):
        ref = CavityOracle(n, re, workers=-1)
        ref.step(steps)
        ep = np.max(np.abs(fields[k][0] - ref.psi)) / np.max(np.abs(ref.psi))
        ew = np.max(np.abs(fields[k][1] - ref.omega)) / np.max(np.abs(ref.omega))
        print(f"  {n}^2 Re {re:g}: psi_rel={ep:.3e} omega_rel={ew:.3e}")
        assert ep <= 1e-11 and ew <= 1e-11, (k, ep, ew)


@pytest.mark.parametrize("members,mode", [(SMALL4, "persistent"), (SMALL4, "graph"),
                                          (SWEEP6, "graph")])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_default_tuning_bitwise_equals_solo(cm, members, mode, precision):
    """The batch's own default tuning (tiles, sweeps per round, check spacing,
    FP32 rounds), each member stopping on its own: on cavities of 130 to 512
    nodes a side (64 x 32 tiles, four sweeps per round) and on the six-cavity
    Reynolds sweep (84 x 54 tiles, five sweeps per round; 981 tiles on a
    co-resident grid of one block per CU, so blocks take several tiles per
    round), every step of every member equals the same cavity run alone with
    the same sweep schedule, bitwise."""
    steps = 3
    print(f"[batch default {mode} precision={precision}] {members}", flush=True)
    c = cm.Cavity([cm.Params(n=n, re=re, precision=precision) for re, n in members])
    c.set_exec(cm.CAVITY_EXEC_PERSISTENT if mode == "persistent" else cm.CAVITY_EXEC_GRAPH)
    bt = c.tuning(-1)
    tiles = sum(((n + bt["tile_x"] - 1) // bt["tile_x"]) * ((n + bt["tile_y"] - 1) // bt["tile_y"])
                for _, n in members)
    print(f"  batch tuning {bt}, {tiles} FP64 tiles")
    solos = []
    for re, n in members:
        s = cm.Cavity(cm.Params(n=n, re=re, precision=precision))
        t = s.tuning()
        # the results do not depend on the tile shape, only on the sweeps per
        # check (FP64) or per refinement round (mixed) and the relaxation
        tx, ty, nt = SOLO_TILES[bt["sweeps_per_launch"]]
        s.set_tuning(tile_x=tx, tile_y=ty, sweeps_per_launch=bt["sweeps_per_launch"], threads=nt,
                     tile_x32=bt["tile_x32"], tile_y32=bt["tile_y32"],
                     sweeps_per_launch32=bt["sweeps_per_launch32"], threads32=bt["threads32"],
                     check_every=bt["check_every"], inner_sweeps=bt["inner_sweeps"],
                     sor_omega=t["sor_omega"])
        solos.append(s)
    for step in range(steps):
        stats = c.step(1)
        for k, solo in enumerate(solos):
            st = solo.step(1)[0]
            p, w, _, _ = solo.fields()
            gp, gw, _, _ = c.fields(k)
            assert np.array_equal(gp, p), (step, k)
            assert np.array_equal(gw, w), (step, k)
            assert stats[k]["sweeps_last_step"] == st["sweeps_last_step"], (step, k)
            assert stats[k]["status"] == 0
    c.close()
    for solo in solos:
        solo.close()
