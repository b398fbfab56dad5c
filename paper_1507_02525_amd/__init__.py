"""MI355X-native multiresolution DFT (MrDFT) — Python binding of libmrdft.so.

The transform (Section 2, eq. (1)): for a signal of N = 2^m samples, level
i = 1..m is the 2^i-point DFT of every non-overlapping length-2^i window,
m*N complex outputs in total, computed on the GPU with the level-reuse
recurrence of Section 3, eq. (4).

Importing this package does not load the GPU library; the compute entry
points (``forward``, ``adjoint``, ``mrdft``, ``spectral_loss``, ``Plan``) do,
and raise ``RuntimeError`` if ``libmrdft.so`` has not been built.  The seeded
input generators live in :mod:`paper_1507_02525_amd.workloads`.
"""
from __future__ import annotations

__all__ = ["Plan", "forward", "adjoint", "mrdft", "MrDFT", "spectral_loss", "SpectralLoss",
           "spectral_loss_terms", "get_plan", "build"]


def build():
    from .build import build as _b
    return _b()


def __getattr__(name):
    if name in ("Plan", "forward", "adjoint", "mrdft", "MrDFT", "spectral_loss", "SpectralLoss",
                "spectral_loss_terms", "get_plan"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
