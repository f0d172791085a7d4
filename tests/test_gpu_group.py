"""Batched multi-unit launches (one persistent sampling kernel for many
(instance, beta, size) units, captured in a HIP graph): each unit's output must
equal the same model sampled on its own, and its statistics the oracle's."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import estimator, physics
from tests.gpu_util import FP32, SPLIT, lattice_cfg, say, to_np
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
            m = fv.Model(cfg, batch + 8, prec, theta)
            units.append(dict(model=m, couplings=fv.couplings(inst), beta=beta, batch=batch - 3 * k, seed=99,
                              stream_id=1000 + k, inst=inst, theta=theta, cfg=cfg))
            k += 1
    return units


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_group_equals_single_model_runs(prec):
    units = _units(prec)
    g = fv.Group(units)
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


def test_group_tile_size_is_the_decode_tile():
    """tile_samples: 0 (default) and 32 build the same group; any other size is
    refused with a message naming the supported one."""
    a = _units(FP32, sizes=(4,), betas=(1.0,))
    fv.Group(a, tile_samples=32)
    with pytest.raises(fv.FvanError, match="32"):
        fv.Group(a, tile_samples=16)
