"""fvan_sample_noalloc (sampling with the library's static KV cache, for callers
that cannot allocate device memory) against fvan_sample: same spins and ln q,
bit for bit, on two calls in a row (the second with a smaller batch), with no
change in free device memory; sizes beyond the static cache are refused."""
import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from tests.gpu_util import FP32, SPLIT, lattice_cfg, say
from workloads import ModelConfig, init_params

pytestmark = pytest.mark.gpu


def _kv_bytes_per_sample(cfg, prec):
    P = min(cfg.prefix, cfg.n_spins)
    S = P + min(cfg.window + 1, cfg.n_spins - P)
    return cfg.n_layers * 2 * S * cfg.d_model * (4 if prec == FP32 else 2)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("shape", ["ea2d_L16", "sk16"])
def test_noalloc_sampling_equals_sampling(prec, shape):
    if shape == "ea2d_L16":
        cfg = lattice_cfg(16, 2, 64, 4, 4)
    else:
        cfg = ModelConfig(16, 32, 2, 2).full_causal()
    per = _kv_bytes_per_sample(cfg, prec)
    cap = fv.NOALLOC_KV_BYTES // per
    b1 = min(1024, cap)
    b2 = max(1, b1 // 3 + 5)
    theta = init_params(cfg, 11, "random")
    ref = fv.Model(cfg, b1, prec, theta, workspaces=fv.WS_SAMPLER)
    m = fv.Model(cfg, cap + 8, prec, theta, workspaces=0)       # no KV cache of its own
    dev = torch.device("cuda")
    out = []
    for k, (b, seed, sid) in enumerate(((b1, 21, 3), (b2, 22, 4))):
        say(f"noalloc sampling: shape {shape}, prec {prec}, call {k + 1}, batch {b} (cache holds {cap})")
        s_ref, lq_ref = ref.sample(b, seed, sid)
        s = torch.full((b, cfg.n_spins), 7, dtype=torch.int8, device=dev)
        lq = torch.full((b,), float("nan"), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        m.sample_noalloc(b, seed, sid, s, lq)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        m.status()
        assert free1 == free0, f"free device memory changed: {free0} -> {free1}"
        assert torch.equal(s, s_ref)
        assert np.array_equal(lq.cpu().numpy().view(np.uint32), lq_ref.cpu().numpy().view(np.uint32))
        out.append(s.cpu().numpy())
    assert not np.array_equal(out[0][:b2], out[1])     # the second call drew new samples
    # beyond the static cache: refused on the host, nothing enqueued
    s = torch.empty((cap + 1, cfg.n_spins), dtype=torch.int8, device=dev)
    lq = torch.empty(cap + 1, dtype=torch.float32, device=dev)
    with pytest.raises(fv.FvanError, match="EINVAL"):
        m.sample_noalloc(cap + 1, 1, 1, s, lq)
    ref.close()
    m.close()
