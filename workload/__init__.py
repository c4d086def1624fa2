"""Seeded synthetic inputs shared by the tests, the smoke check and the bench."""
from .gen import (Workload, Client, config, posterior_shell, make, freq_grid,
                  prior_batch, shell_batch, serving_clients, CONFIGS,
                  CONFIG_NAMES, SEED_BASE, T_CMB, NU_REF)

__all__ = ["Workload", "Client", "config", "posterior_shell", "make",
           "freq_grid", "prior_batch", "shell_batch", "serving_clients",
           "CONFIGS", "CONFIG_NAMES", "SEED_BASE", "T_CMB", "NU_REF"]
