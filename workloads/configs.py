"""Link and workload descriptions for the five SSFM workloads.

A :class:`Link` is a flat record of the numbers that define one amplified
fibre link, in the units such links are quoted in (km, dB/km, ps^2/km,
1/(W km), dB).  It carries no derived quantities: the oracle and the HIP
library each convert to SI on their own.

The workloads are:

1. single-pol NLSE, one 80 km SSMF span in 80 steps of 1 km, 4096 samples
   (2048 16-QAM symbols at 32 GBd, 2 samples/symbol), 0 dBm, no amplifier;
2. dual-pol Manakov, 10 x 80 km spans, 100 steps/span, EDFA 16 dB / NF 5 dB
   with ASE, 2^16 samples per pol (64 GBd, 2 sps), +2 dBm total launch;
3. WDM Manakov, 5 x 64 GBd channels on a 75 GHz grid, 2^18 samples per pol,
   20 x 80 km spans, 200 steps/span, EDFA + ASE, 0 dBm per channel;
4. a batch of 256 independent dual-pol realisations with mixed lengths,
   launch powers, span counts and noise seeds (50 steps/span);
5. learned digital back-propagation over a 10 x 80 km received field.

Readings where the workload statement is incomplete or inconsistent:

* workload 3 quotes "4 sps over 375 GHz"; 4 x 64 GBd cannot hold carriers at
  +-150 GHz, and 375 GS/s puts the 75 GHz grid off the FFT bins.  The
  sample rate used is 512 GS/s (8 samples/symbol), which places the five
  carriers on exact bins (k * 38400 at 2^18 points).  The work per step
  depends only on the sample count, so this does not change the cost.
* workload 4 states no symbol rate or span-count law: 64 GBd, 2 sps, and a
  span count uniform on {1..10}.
* workload 5 states no forward step count: 100 steps/span as workload 2.
* the carrier frequency is not stated anywhere: 193.4145 THz (1550 nm).
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = ["Link", "Workload", "CONFIGS", "config_link", "BatchItem",
           "batch_config", "DEFAULT_CARRIER_HZ"]

DEFAULT_CARRIER_HZ = 193.4145e12  # 1550 nm


@dataclass(frozen=True)
class Link:
    """One amplified fibre link, in quoted units.

    ``nl_factor`` NaN selects the default (1 for one polarisation, 8/9 for
    the Manakov equation); ``edfa_gain_db`` 0 means no amplifier gain;
    ``carrier_hz`` NaN selects 193.4145 THz.
    """

    n_pol: int
    n_samples: int
    sample_rate_hz: float
    span_km: float
    n_spans: int
    steps_per_span: int
    alpha_db_per_km: float
    beta2_ps2_per_km: float
    gamma_per_w_km: float
    nl_factor: float = float("nan")
    edfa_gain_db: float = 0.0
    edfa_nf_db: float = 0.0
    ase: bool = False
    carrier_hz: float = float("nan")

    def replace(self, **kw) -> "Link":
        return dataclasses.replace(self, **kw)

    @property
    def total_steps(self) -> int:
        return self.n_spans * self.steps_per_span


@dataclass(frozen=True)
class Workload:
    """A link plus the recipe of its transmitted field."""

    name: str
    link: Link
    symbol_rate_hz: float
    sps: int
    launch_dbm: float            # total over polarisations (per channel for WDM)
    rolloff: float = 0.1
    n_channels: int = 1
    channel_spacing_hz: float = 0.0
    symbol_seed: int = 0
    ase_seed: int = 0


_SSMF = dict(alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7, gamma_per_w_km=1.3)

CONFIGS = {
    1: Workload(
        name="nlse-1x80km-4096",
        link=Link(n_pol=1, n_samples=4096, sample_rate_hz=64e9, span_km=80.0,
                  n_spans=1, steps_per_span=80, **_SSMF),
        symbol_rate_hz=32e9, sps=2, launch_dbm=0.0,
        symbol_seed=20250703 + 1, ase_seed=1001),
    2: Workload(
        name="manakov-10x80km-2^16",
        link=Link(n_pol=2, n_samples=1 << 16, sample_rate_hz=128e9,
                  span_km=80.0, n_spans=10, steps_per_span=100, **_SSMF,
                  edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True),
        symbol_rate_hz=64e9, sps=2, launch_dbm=2.0,
        symbol_seed=20250703 + 2, ase_seed=1002),
    3: Workload(
        name="wdm5-manakov-20x80km-2^18",
        link=Link(n_pol=2, n_samples=1 << 18, sample_rate_hz=512e9,
                  span_km=80.0, n_spans=20, steps_per_span=200, **_SSMF,
                  edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True),
        symbol_rate_hz=64e9, sps=8, launch_dbm=0.0,
        n_channels=5, channel_spacing_hz=75e9,
        symbol_seed=20250703 + 3, ase_seed=1003),
    5: Workload(
        name="ldbp-64x2^14-10x80km",
        link=Link(n_pol=2, n_samples=1 << 14, sample_rate_hz=128e9,
                  span_km=80.0, n_spans=10, steps_per_span=100, **_SSMF,
                  edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True),
        symbol_rate_hz=64e9, sps=2, launch_dbm=2.0,
        symbol_seed=20250703 + 5, ase_seed=1005),
}


def config_link(i: int) -> Link:
    return CONFIGS[i].link


@dataclass(frozen=True)
class BatchItem:
    """One realisation of the batched workload (workload 4)."""

    n_samples: int
    launch_dbm: float
    n_spans: int
    seed: int
    symbol_seed: int

    def link(self) -> Link:
        return Link(n_pol=2, n_samples=self.n_samples, sample_rate_hz=128e9,
                    span_km=80.0, n_spans=self.n_spans, steps_per_span=50,
                    **_SSMF, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


def batch_config(n: int = 256, seed: int = 20250703 + 4,
                 lengths=(1 << 12, 1 << 13, 1 << 14, 1 << 15, 1 << 16)
                 ) -> List[BatchItem]:
    """Workload 4: ``n`` realisations with lengths drawn from ``lengths``,
    launch power uniform in [-4, +6] dBm, 1..10 spans, distinct seeds."""
    rng = np.random.default_rng(seed)
    ln = rng.choice(np.asarray(lengths, dtype=np.int64), size=n)
    p = rng.uniform(-4.0, 6.0, size=n)
    spans = rng.integers(1, 11, size=n)
    return [BatchItem(n_samples=int(ln[i]), launch_dbm=float(p[i]),
                      n_spans=int(spans[i]), seed=4000 + i,
                      symbol_seed=seed * 1000 + i) for i in range(n)]


@dataclass(frozen=True)
class LdbpConfig:
    """Workload 5's learned back-propagation: ``batch`` received fields of
    the workload-5 link, K = n_spans * steps_per_span FIR + Kerr steps of
    ``n_taps`` taps, loss through a ``2 mf_half + 1``-tap RRC matched filter
    at the workload's samples per symbol."""

    workload: Workload
    batch: int = 64
    n_taps: int = 15
    steps_per_span: int = 2
    mf_half: int = 64

    @property
    def n_steps(self) -> int:
        return self.workload.link.n_spans * self.steps_per_span


LDBP = LdbpConfig(workload=CONFIGS[5])
