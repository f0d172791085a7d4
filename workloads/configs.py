"""Model and workload descriptions (sizes only).

The five workloads mirror the ones the method is exercised on: a small SK model
that exact enumeration can check, a periodic 2D Edwards-Anderson lattice with
+/-J bonds, a large dense SK model, a periodic 3D Edwards-Anderson lattice with
Gaussian bonds, and a batch of many 2D instances at several temperatures.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple


@dataclass(frozen=True)
class ModelConfig:
    """Shape of the autoregressive transformer.

    window / prefix describe the attention mask: key position j is visible from
    query position t iff j <= t and (t - j <= window or j < prefix).  They are
    normally derived from the interaction graph; -1 means "not yet derived".
    """
    n_spins: int
    d_model: int
    n_layers: int
    n_heads: int
    d_token: int = 2
    vocab: int = 2
    window: int = -1
    prefix: int = 0

    @property
    def d_pos(self) -> int:
        return self.d_model - self.d_token

    @property
    def d_head(self) -> int:
        return self.d_model // self.n_heads

    def with_mask(self, window: int, prefix: int) -> "ModelConfig":
        return replace(self, window=int(window), prefix=int(prefix))

    def full_causal(self) -> "ModelConfig":
        return replace(self, window=self.n_spins - 1, prefix=0)


@dataclass(frozen=True)
class Workload:
    name: str
    model: ModelConfig
    batch: int
    kind: str                      # "sk" | "ea"
    size: int                      # N for SK, L for EA
    dim: int = 0                   # lattice dimension for EA
    bonds: str = "gauss"           # "gauss" | "pm1"
    betas: Tuple[float, ...] = (1.0,)
    pbc: bool = True
    instance_seed: int = 0
    param_seed: int = 0
    sizes: Tuple[int, ...] = field(default_factory=tuple)   # batched workload: L values
    n_instances: int = 1


def _w(idx: int, **kw) -> Workload:
    return Workload(instance_seed=1000 * idx, param_seed=7 * idx, **kw)


WORKLOADS = {
    "sk16": _w(1, name="sk16", model=ModelConfig(16, 32, 2, 2), batch=1024,
               kind="sk", size=16, betas=(1.0,)),
    "ea2d_L16": _w(2, name="ea2d_L16", model=ModelConfig(256, 64, 4, 4), batch=4096,
                   kind="ea", size=16, dim=2, bonds="pm1", betas=(0.5, 1.0, 2.0)),
    "sk512": _w(3, name="sk512", model=ModelConfig(512, 128, 6, 8), batch=8192,
                kind="sk", size=512, betas=(1.5,)),
    "ea3d_L10": _w(4, name="ea3d_L10", model=ModelConfig(1000, 128, 8, 8), batch=16384,
                   kind="ea", size=10, dim=3, bonds="gauss", betas=(0.5, 1.0, 2.0)),
    "ea2d_batched": _w(5, name="ea2d_batched", model=ModelConfig(1024, 64, 4, 4), batch=1024,
                       kind="ea", size=32, dim=2, bonds="pm1",
                       betas=tuple(0.2 + 0.4 * k for k in range(8)),
                       sizes=(16, 24, 32), n_instances=64),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
