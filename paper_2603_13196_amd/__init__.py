"""MI355X-native batched Gaussian log-likelihood of the region-based 21-cm
foreground model (Tutt et al.; Eqs. fast_forward_model, t21model, likelihood).

The computation lives in the HIP library ``libfgl.so`` (C-ABI in
include/fgl.h); ``paper_2603_13196_amd.fgl`` is its ctypes binding and fails
on import if the library is not built.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfgl.so")


def load():
    """Import and return the binding module (raises ImportError if unbuilt)."""
    from . import fgl
    return fgl
