"""Seeded synthetic TPC time frames (inputs only; no reconstruction arithmetic)."""
from .generator import (Frames, Tracks, make_frames, make_config, config_params, make_row_x,
                        sector_alpha, sector_side, CONFIG_NAMES, C_LIGHT, TAN10, drop_clusters, add_clusters,
                        make_scattering_frame, highland_theta0, PION_MASS, PROTON_MASS, ARGON_GAS, TPC_GAS,
                        mean_dedx)

__all__ = ["Frames", "Tracks", "make_frames", "make_config", "config_params", "make_row_x",
           "sector_alpha", "sector_side", "CONFIG_NAMES", "C_LIGHT", "TAN10", "drop_clusters", "add_clusters", "make_scattering_frame", "highland_theta0",
           "PION_MASS", "PROTON_MASS", "ARGON_GAS", "TPC_GAS", "mean_dedx"]
