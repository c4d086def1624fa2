"""Seeded synthetic inputs shared by the tests, the smoke check and the bench."""
from .gen import (Workload, Client, config, posterior_shell, make, freq_grid,
                  prior_batch, shell_batch, serving_clients, WORKLOADS,
                  SMALL, MEDIUM, HEADLINE, LARGE, SEED_BASE, T_CMB, NU_REF, make_masks,
                  masks_config, MASKS_NAME, PRIOR_ALPHA)

__all__ = ["Workload", "Client", "config", "posterior_shell", "make",
           "freq_grid", "prior_batch", "shell_batch", "serving_clients",
           "WORKLOADS", "SMALL", "MEDIUM", "HEADLINE", "LARGE", "SEED_BASE", "T_CMB", "NU_REF",
           "make_masks", "masks_config", "MASKS_NAME", "PRIOR_ALPHA"]
