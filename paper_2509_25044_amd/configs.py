"""The five workload configurations (shapes, loss settings, iteration counts).

Shapes follow the paper's workloads: a 64^3 toy pair, the clinical 1 mm
brain shape 160x192x224, a 512^3 pair at 250 um-like scale and one GPU's
share (1024^3 plus an 8-voxel halo) of the 100 um gigavoxel problem of the
paper's large-scale experiment.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

from .synth import PairSpec


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    pair: PairSpec
    roi: Optional[Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, int]]]  # ((z0,z1),(y0,y1),(x0,x1))
    lncc_window: int = 5
    lncc_eps: float = 1e-5
    mi_bins: int = 32
    iters: int = 50
    lr: float = 0.1
    levels: Tuple[float, ...] = (1.0,)

    @property
    def shape(self):
        return self.pair.shape

    @property
    def n_roi(self) -> int:
        if self.roi is None:
            D, H, W = self.shape
            return D * H * W
        return (self.roi[0][1] - self.roi[0][0]) * (self.roi[1][1] - self.roi[1][0]) * (self.roi[2][1] - self.roi[2][0])


C1 = Workload("c1_64cube_lncc5", PairSpec((64, 64, 64), (3.0, 8.0), 3.0), None,
              lncc_window=5, iters=50, lr=0.1)
C2 = Workload("c2_clinical_160x192x224_mi32_lncc7",
              PairSpec((160, 192, 224), (4.0, 12.0), 3.0, multimodal=True), None,
              lncc_window=7, mi_bins=32, iters=200, lr=0.1, levels=(0.25, 0.5, 1.0))
C3 = Workload("c3_512cube_lncc5_mi32", PairSpec((512, 512, 512), (3.0, 8.0), 8.0), None,
              lncc_window=5, mi_bins=32, iters=300, lr=0.1)
C5 = Workload("c5_1024cube_halo8_lncc5_mi32",
              PairSpec((1040, 1040, 1040), (10.0, 40.0), 8.0, texture_std=0.05), ((8, 1032),) * 3,
              lncc_window=5, mi_bins=32, iters=100, lr=0.1)

ALL = {w.name: w for w in (C1, C2, C3, C5)}
