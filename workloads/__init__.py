"""Seeded synthetic inputs for the SSFM path.

This package generates the *inputs* that both the FP64 oracle and the HIP
library consume: link descriptions (plain numbers in the units a link is
usually quoted in) and transmitted optical fields (16-QAM, root-raised-cosine
shaping, launch-power normalisation, WDM multiplexing).  It holds none of the
propagation arithmetic: no dispersion, nonlinearity, amplifier or noise model
lives here, so the oracle and the GPU path stay independent of each other.
"""

from .configs import Link, CONFIGS, config_link, BatchItem, batch_config, LdbpConfig, LDBP
from .signals import (qam16_symbols, rrc_response, rrc_taps, shaped_field,
                      dual_pol_field, wdm_field, make_field, dbm_to_watt,
                      field_and_targets)

__all__ = [
    "Link", "CONFIGS", "config_link", "BatchItem", "batch_config",
    "qam16_symbols", "rrc_response", "rrc_taps", "shaped_field",
    "dual_pol_field", "wdm_field", "make_field", "dbm_to_watt",
    "field_and_targets", "LdbpConfig", "LDBP",
]
