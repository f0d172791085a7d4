"""Batched multi-unit launches (one persistent sampling kernel for many
(instance, beta, size) units, captured in a HIP graph): each unit's output must
equal the same model sampled on its own, and its statistics the oracle's."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import estimator, network as net, philox, physics
from tests.gpu_util import DECISION_TOL, FP32, SITE_TOL, SPLIT, lattice_cfg, say, to_np
from workloads import ea_instance, init_params

pytestmark = pytest.mark.gpu


def _units(prec, sizes=(4, 6, 8), betas=(0.5, 1.5), batch=40, d=64):
    units = []
    k = 0
    for L in sizes:
        cfg = lattice_cfg(L, 2, d, 2, 4)
        for beta in betas:
            inst = ea_instance(L, 2, 500 + k, "pm1")
            theta = init_params(cfg, 10 + k, "random")
            m = fv.Model(cfg, batch + 8, prec, theta, workspaces=fv.WS_SAMPLER)
            units.append(dict(model=m, couplings=fv.couplings(inst), beta=beta, batch=batch - 3 * k, seed=99,
                              stream_id=1000 + k, inst=inst, theta=theta, cfg=cfg))
            k += 1
    return units


@pytest.mark.parametrize("tile", [0, 16, 32])
@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_group_equals_single_model_runs(prec, tile):
    """Every tile shape (0: the autotuner's choice) gives each unit exactly the
    samples of its model sampled alone (the per-sample arithmetic does not depend
    on the tile)."""
    units = _units(prec)
    g = fv.Group(units, tile_samples=tile)
    say(f"group launch shape {g.launch_shape()}")
    if tile:
        assert g.launch_shape()["tile"] == tile
    g.run()
    torch.cuda.synchronize()
    for u, out in zip(units, g.outputs):
        s, lq = u["model"].sample(u["batch"], u["seed"], u["stream_id"])
        E = fv.energy(u["couplings"], s)
        st = fv.free_energy(E, lq, u["beta"], u["cfg"].n_spins)
        torch.cuda.synchronize()
        assert torch.equal(out["spins"], s)
        assert torch.equal(out["log_q"], lq)
        assert torch.equal(out["energy"], E)
        Eref = physics.energy_edges_int(to_np(s), u["inst"].edges_i, u["inst"].edges_j, u["inst"].J)
        assert np.array_equal(to_np(out["energy"]).astype(np.int64), Eref)
        mean, var = estimator.free_energy_stats(Eref, to_np(lq).astype(np.float64), u["beta"], u["cfg"].n_spins)
        got = to_np(out["stats"])
        assert abs(got[0] - mean) <= 1e-12 * abs(mean) and abs(got[1] - var) <= 1e-9 * var + 1e-300
        assert np.array_equal(got, to_np(st))


def test_group_graph_replays_match_eager():
    units = _units(FP32, sizes=(5, 7), betas=(1.0,), batch=33)
    g = fv.Group(units)
    g.run()
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in g.outputs]
    for rep in range(3):
        for o in g.outputs:          # clobber the outputs with eager work between replays
            o["spins"].zero_()
            o["stats"].fill_(7.0)
        torch.cuda.synchronize()
        g.run_graph()
        torch.cuda.synchronize()
        for o, r in zip(g.outputs, ref):
            for k in r:
                assert torch.equal(o[k], r[k]), (rep, k)


def test_group_rejects_mismatched_models():
    a = _units(FP32, sizes=(4,), betas=(1.0,))
    cfg = lattice_cfg(4, 2, 32, 2, 2)
    m = fv.Model(cfg, 40, FP32, init_params(cfg, 1))
    a.append(dict(model=m, couplings=a[0]["couplings"], beta=1.0, batch=10, seed=1, stream_id=1))
    with pytest.raises(fv.FvanError):
        fv.Group(a)
    b = _units(FP32, sizes=(4,), betas=(1.0,))
    b.append(dict(b[0]))
    with pytest.raises(fv.FvanError):
        fv.Group(b)


def test_group_tile_sizes():
    """tile_samples 0 (autotuned), 16 and 32 are accepted; any other size is
    refused with a message naming the supported ones."""
    a = _units(FP32, sizes=(4,), betas=(1.0,))
    for t in (0, 16, 32):
        fv.Group(a, tile_samples=t).close()
    with pytest.raises(fv.FvanError, match="16 or 32"):
        fv.Group(a, tile_samples=8)


_REUSE_SCRIPT = """
import json, sys, torch
sys.path.insert(0, {root!r})
import paper_2606_22984_amd as fv
from tests.gpu_util import lattice_cfg
from workloads import ea_instance, init_params
units = []
for k, L in enumerate((6, 8)):
    cfg = lattice_cfg(L, 2, 64, 2, 4)
    m = fv.Model(cfg, 200, fv.FVAN_BF16_SPLIT, init_params(cfg, k), workspaces=fv.WS_SAMPLER)
    units.append(dict(model=m, couplings=fv.couplings(ea_instance(L, 2, k, "pm1")), beta=1.0, batch=200, seed=1,
                      stream_id=k))
g = fv.Group(units)
print(json.dumps(g.launch_shape()))
"""


def test_group_launch_shape_is_persisted_and_reused(tmp_path):
    """A second process building a group of the same shape takes the first one's
    tuned launch shape from the store, without timing."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, FVAN_TUNE_FILE=str(tmp_path / "tune.json"))
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", _REUSE_SCRIPT.format(root=root)], env=env, capture_output=True,
                           text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    say(f"first process {outs[0]}, second {outs[1]}")
    assert not outs[0]["from_store"] and outs[1]["from_store"]
    assert (outs[0]["tile"], outs[0]["grid"]) == (outs[1]["tile"], outs[1]["grid"])
    store = (tmp_path / "tune.json").read_text()
    assert '"tile": %d, "grid": %d' % (outs[0]["tile"], outs[0]["grid"]) in store


@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_group_matches_oracle_at_batched_workload_shape(prec, tile):
    """The batched workload's unit shape (2D EA, d_model 64, 4 layers, 4 heads,
    1024 samples per unit) at L = 16, 24 and 32 in one group, each unit checked
    against the FP64 oracle directly: the teacher-forced decision check and the
    per-site ln q on rows of the first tile, both sides of a tile boundary and
    the last tile; energies exact and F_q statistics against the oracle."""
    B = 1024
    units = []
    for k, L in enumerate((16, 24, 32)):
        inst = ea_instance(L, 2, 900 + k, "pm1")
        cfg = lattice_cfg(L, 2, 64, 4, 4)
        assert (cfg.window, cfg.prefix) == (L, L + 1)
        theta = init_params(cfg, 40 + k, "default")
        m = fv.Model(cfg, B, prec, theta, workspaces=fv.WS_SAMPLER)
        units.append(dict(model=m, couplings=fv.couplings(inst), beta=0.2 + 1.4 * k, batch=B, seed=17,
                          stream_id=300 + k, inst=inst, theta=theta, cfg=cfg))
    g = fv.Group(units, tile_samples=tile)
    g.run_graph()
    torch.cuda.synchronize()
    rows = [0, 15, 16, 31, 32, 500, B - 1]
    for u, out in zip(units, g.outputs):
        cfg = u["cfg"]
        say(f"group unit L={int(round(cfg.n_spins ** 0.5))} prec {prec}: oracle on rows {rows}")
        sp = to_np(out["spins"])
        lq = to_np(out["log_q"]).astype(np.float64)
        assert set(np.unique(sp)).issubset({-1, 1}) and np.all(np.isfinite(lq))
        sub = sp[rows]
        th = net.as_theta(u["theta"])
        pp = net.cond_plus(th, cfg, sub, chunk=8).numpy()
        uu = np.concatenate([philox.uniforms(u["seed"], u["stream_id"], 1, cfg.n_spins, b) for b in rows])
        wrong = (uu < pp) != (sub > 0)
        gap = np.abs(uu - pp)
        bad = int((wrong & (gap >= DECISION_TOL[prec])).sum())
        say(f"  decision mismatches outside tol {bad}, inside {int(wrong.sum()) - bad}")
        assert bad == 0
        ref = net.log_q(th, cfg, sub, chunk=8).numpy()
        per_site = np.abs(lq[rows] - ref) / cfg.n_spins
        say(f"  max per-site |d ln q| {per_site.max():.3e}")
        assert per_site.max() <= SITE_TOL[prec]
        Eref = physics.energy_edges_int(sp, u["inst"].edges_i, u["inst"].edges_j, u["inst"].J)
        assert np.array_equal(to_np(out["energy"]).astype(np.int64), Eref)
        mean, var = estimator.free_energy_stats(Eref, lq, u["beta"], cfg.n_spins)
        st = to_np(out["stats"])
        assert abs(st[0] - mean) <= 1e-12 * abs(mean) and abs(st[1] - var) <= 1e-9 * var


def test_group_gaussian_bond_energies_equal_single_kernel():
    """Float (Gaussian) bonds: the group's energy kernel sums in the single-model
    kernel's order, so its energies equal fvan_energy's bitwise."""
    units = []
    for k, L in enumerate((4, 6)):
        cfg = lattice_cfg(L, 2, 32, 2, 2)
        inst = ea_instance(L, 2, 70 + k, "gauss")
        m = fv.Model(cfg, 48, FP32, init_params(cfg, 3 + k, "random"), workspaces=fv.WS_SAMPLER)
        units.append(dict(model=m, couplings=fv.couplings(inst), beta=1.0, batch=45, seed=2, stream_id=k,
                          inst=inst))
    g = fv.Group(units)
    g.run()
    torch.cuda.synchronize()
    for u, out in zip(units, g.outputs):
        E = fv.energy(u["couplings"], out["spins"])
        torch.cuda.synchronize()
        assert out["energy"].dtype == torch.float32
        assert torch.equal(out["energy"], E)
        ref = physics.energy_edges(to_np(out["spins"]), u["inst"].edges_i, u["inst"].edges_j,
                                   u["inst"].J.astype(np.float32).astype(np.float64))
        assert np.max(np.abs(to_np(E).astype(np.float64) - ref)) <= 1e-5 * u["inst"].n
