"""Batched D2Q9 simulations: one launch per phase over all members, the step
replayed from a hipGraph.  Every member must give, bit for bit, the results
of the same simulation created alone (and so the oracle's, to the parity
bar of the single path)."""
import numpy as np
import pytest

from paper_1906_03065_amd import lbib
from paper_1906_03065_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mixed(count=7, seed=11):
    """Capsule-at-interface runs of uneven sizes over all three size classes,
    plus one without a membrane (a flat interface)."""
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(g.choice([80, 96, 112, 144, 200, 272, 320]))
        ny = n + int(g.integers(-8, 9))
        # the tile map (r_cut + 1 = 18 around the capsule) must fit in the
        # period: 2 R + 36 < n (kept at 2 R + 40)
        R = float(g.uniform(8.0, min(0.25 * min(n, ny), (n - 41) / 2.0)))
        nm = int(min(384, max(64, np.ceil(2 * np.pi * R / 0.8))))
        kap = g.uniform(0.01, 0.05, 3)
        w = W.capsule_at_interface(nx=n, ny=ny, R=R, n_markers=nm, kappa=kap, kappa_s=float(10 ** g.uniform(-3, -1)),
                                   kappa_b=float(10 ** g.uniform(-5, -3)), wall_y=1, perturb=1e-4,
                                   seed=100 + k)
        out.append(w)
    f = W.flat(nx=40, ny=64)
    out.append(f)
    return out


def _single(w):
    return lbib.from_workload(w, storage="fp32")


def _same(a, b):
    fa, fb = a.fields(), b.fields()
    for k in fa:
        if not np.array_equal(fa[k], fb[k]):
            return False, k, float(np.abs(fa[k] - fb[k]).max())
    for i in range(len(a.mem_sizes)):
        ma, mb = a.membrane(i), b.membrane(i)
        for q in ("X", "U", "F"):
            if not np.array_equal(ma[q], mb[q]):
                return False, f"{q}{i}", float(np.abs(ma[q] - mb[q]).max())
    return True, None, 0.0


@pytest.mark.parametrize("graph", [1, 0])
def test_batch_equals_single_runs(graph):
    """Eight uneven members (three size classes, one with no membrane), 60
    steps, graph replay on or off: every member bitwise equal to its single
    run."""
    ws = _mixed()
    b = lbib.Batch.from_workloads(ws)
    b.graph(graph)
    b.step(60)
    b.synchronize()
    assert b.graph() == graph
    assert b.check() == 0
    for k, w in enumerate(ws):
        s = _single(w)
        s.step(60)
        ok, key, err = _same(b[k], s)
        print(k, w["name"], ok, key, err, flush=True)
        assert ok, (k, key, err)
        assert b[k].steps_done == 60


@pytest.mark.parametrize("form", [0, 1])
def test_batch_members_vs_oracle(orc, form):
    """An uneven FP32 batch (one member in each size class: lattice widths
    96, 200 and 300, tau != 1 in one of them) stepped 500 times, in the
    potential (form 0) or divergence (form 1) force form: every member
    against the FP64 oracle, field by field, within the FP32 bar of 1e-5,
    and its markers within 1e-4."""
    from helpers import compare, marker_err, run_oracle

    ws = [W.capsule_at_interface(nx=96, ny=88, R=14.0, n_markers=110, kappa=(0.02, 0.03, 0.015), seed=31),
          W.capsule_at_interface(nx=200, ny=72, R=12.5, n_markers=98, kappa=(0.03, 0.02, 0.025), tau=0.8,
                                 tau_phi=1.3, seed=32, kappa_s=0.05, kappa_b=1e-3),
          W.capsule_at_interface(nx=300, ny=64, R=11.0, n_markers=88, centre=(83.4, 31.7), seed=33)]
    for w in ws:
        w["params"]["force_form"] = form
    b = lbib.Batch.from_workloads(ws)
    assert sorted(b.get_launch(c)["members"] for c in range(3)) == [1, 1, 1]
    b.step(500)
    b.synchronize()
    for k, w in enumerate(ws):
        o = run_oracle(orc, w)
        o.step(500)
        errs = compare(b[k], o)
        dx = marker_err(b[k], o, 1)
        print(f"form {form} member {k} {w['params']['nx']}x{w['params']['ny']}",
              {q: f"{v:.2e}" for q, v in errs.items()}, f"markers {dx:.2e}", flush=True)
        for q, v in errs.items():
            assert v <= 1e-5, (k, q, v)
        assert dx < 1e-4, (k, dx)


def test_batch_launch_shapes_bitwise():
    """Other lanes per workgroup, rows per item and ring depths per size
    class change nothing in the results."""
    ws = _mixed(count=5, seed=3)
    ref = lbib.Batch.from_workloads(ws)
    ref.step(25)
    alt = lbib.Batch.from_workloads(ws)
    alt.set_launch(0, block_x=128, seg=7, ring=4)
    alt.set_launch(1, block_x=64, seg=13, ring=3)
    alt.set_launch(2, block_x=128, seg=-1, ring=4)
    alt.step(25)
    for k in range(len(ws)):
        ok, key, err = _same(ref[k], alt[k])
        assert ok, (k, key, err)
    for c in range(3):
        print(c, alt.get_launch(c), flush=True)


def test_batch_state_rules():
    """Members step only with their batch; per-simulation calls on the batch
    handle are refused; D3Q19 members are refused."""
    ws = _mixed(count=2, seed=5)
    b = lbib.Batch.from_workloads(ws)
    with pytest.raises(lbib.LbibError) as e:
        b[0].step(1)
    assert e.value.code == lbib.ESTATE
    assert lbib.lib().lbib_step(b.h, 3) == 0  # odd: every member now reads buffer B
    assert lbib.lib().lbib_energy(b.h, None) == lbib.EINVAL
    p3 = W.base_params(16, 16, 16, lattice=1)
    with pytest.raises(lbib.LbibError):
        lbib.Batch([p3])
    # a member whose fields are set again restarts alone: the batch refuses
    # to step until the parities agree
    f = ws[0]["fields"]
    b[0].set_fields(f["rho"], f["phi"], f["psi"])
    assert lbib.lib().lbib_step(b.h, 1) == lbib.ESTATE
