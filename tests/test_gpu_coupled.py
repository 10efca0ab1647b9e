"""GPU parity of the coupled mode (fixed relaxation sweeps per stage) against
the FP64 oracle, through the C ABI.

Tolerance 1e-11 relative in psi and omega, as for the solved mode.  Also:
the number of sweeps per kernel launch does not change the result (bitwise),
including sweep counts that leave a remainder; the mode's restrictions; a
blow-up is reported.
"""
import numpy as np
import pytest

from oracle.cavity_oracle import CavityOracle

pytestmark = pytest.mark.gpu

PARITY = 1e-11


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0809_3098_amd.cavity as cav
    return cav


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n,re,m,beta,steps", [(64, 1000.0, 10, 0.8, 100), (257, 1e4, 8, 0.5, 10),
                                               (1024, 1e4, 6, 0.8, 2), (33, 400.0, 7, 0.1, 40)])
def test_coupled_parity(cm, n, re, m, beta, steps):
    print(f"[coupled parity] n={n} re={re} sweeps={m} beta={beta} steps={steps}", flush=True)
    c = cm.Cavity(cm.Params(n=n, re=re, fixed_sweeps=m, sor_omega=beta))
    st = c.step(steps)[0]
    psi, omega, _, _ = c.fields()
    c.close()
    ref = CavityOracle(n, re, fixed_sweeps=m, beta=beta, workers=-1)
    d = ref.step(steps, diagnostics_every=steps)
    ep, ew = _rel(psi, ref.psi), _rel(omega, ref.omega)
    print(f"  psi_rel={ep:.3e} omega_rel={ew:.3e}")
    assert ep <= PARITY and ew <= PARITY, (ep, ew)
    assert st["sweeps_last_step"] == 5 * m and st["status"] == 0
    assert st["ke"] == pytest.approx(d["ke"], rel=1e-9)


@pytest.mark.parametrize("m", [6, 7, 8])
def test_sweeps_per_launch_do_not_change_the_result(cm, m):
    n, re, steps = 200, 5000.0, 4
    print(f"[coupled launch split] n={n} sweeps={m}", flush=True)
    out = []
    for tx, ty, s, nt in ((64, 64, 4, 1024), (64, 64, 3, 1024), (32, 32, 1, 256)):
        c = cm.Cavity(cm.Params(n=n, re=re, fixed_sweeps=m, sor_omega=0.6))
        c.set_tuning(tile_x=tx, tile_y=ty, sweeps_per_launch=s, threads=nt, xcd_bands=0)
        c.step(steps, want_stats=False)
        out.append(c.fields()[:2])
        c.close()
    for p, w in out[1:]:
        assert np.array_equal(p, out[0][0]) and np.array_equal(w, out[0][1])


def test_coupled_restrictions_and_batch(cm):
    print("[coupled restrictions]", flush=True)
    members = [(1000.0, 64), (3000.0, 97)]
    c = cm.Cavity([cm.Params(n=n, re=re, fixed_sweeps=5, sor_omega=0.7) for re, n in members])
    assert c.exec_mode() == cm.CAVITY_EXEC_STREAM
    with pytest.raises(cm.CavityError) as e:
        c.set_exec(cm.CAVITY_EXEC_PERSISTENT)
    assert e.value.code == cm.CAVITY_EINVAL
    with pytest.raises(cm.CavityError) as e:
        c.set_tuning(0, solver=cm.CAVITY_SOLVER_MG)
    assert e.value.code == cm.CAVITY_EINVAL
    c.step(3, want_stats=False)
    got = [c.fields(k)[:2] for k in range(2)]
    c.close()
    for k, (re, n) in enumerate(members):
        s = cm.Cavity(cm.Params(n=n, re=re, fixed_sweeps=5, sor_omega=0.7))
        s.step(3, want_stats=False)
        p, w = s.fields()[:2]
        s.close()
        assert np.array_equal(got[k][0], p) and np.array_equal(got[k][1], w)
    # a handle mixing coupled and solved cavities has no graph execution
    c = cm.Cavity([cm.Params(n=64, re=1000.0, fixed_sweeps=5), cm.Params(n=64, re=1000.0)])
    with pytest.raises(cm.CavityError) as e:
        c.set_exec(cm.CAVITY_EXEC_GRAPH)
    assert e.value.code == cm.CAVITY_EINVAL
    c.close()


def test_coupled_graph_replays_equal_stream_steps(cm):
    """Every replay (host work and a tuning change in between) is compared."""
    members = [(2000.0, 130), (8000.0, 257)]
    steps = 5
    print(f"[coupled graph] {members}", flush=True)
    mk = lambda: cm.Cavity([cm.Params(n=n, re=re, fixed_sweeps=9, sor_omega=0.6)
                            for re, n in members])
    g, s = mk(), mk()
    g.set_exec(cm.CAVITY_EXEC_GRAPH)
    for step in range(steps):
        if step == 3:  # new relaxation: the captured graphs must not be reused
            for c in (g, s):
                c.set_tuning(1, sor_omega=0.4)
        sg, ss = g.step(1), s.step(1)
        for k in range(len(members)):
            pg, wg = g.fields(k)[:2]
            ps, ws = s.fields(k)[:2]
            assert np.array_equal(pg, ps) and np.array_equal(wg, ws), (step, k)
            assert sg[k]["sweeps_last_step"] == ss[k]["sweeps_last_step"] == 45
            assert sg[k]["last_resid_inf"] == ss[k]["last_resid_inf"]
    g.close()
    s.close()


def test_coupled_blow_up_is_detected(cm):
    print("[coupled nonfinite]", flush=True)
    c = cm.Cavity(cm.Params(n=33, re=1.0e6, cfl=40.0, fixed_sweeps=4, sor_omega=0.8))
    with pytest.raises(cm.CavityError) as e:
        c.step(400, want_stats=False)
    assert e.value.code == cm.CAVITY_ENONFINITE
    c.close()
