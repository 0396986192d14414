"""QEM E-step hot path for AMD MI355X (gfx950).

``libqem.so`` (HIP kernels behind the C ABI of include/qem.h) runs massively
parallel importance weighting, its log-space contraction, the reverse pass,
moments and the EMA/M-step of QEM (arXiv 2503.08264, section 3.2 and
Algorithm 1).  ``api.QEM`` is the thin Python binding; ``autograd`` wraps the
contraction as a torch.autograd.Function; ``encoder`` holds the amortised
initialiser of the proposal.
"""
from ._lib import QEMError, load  # noqa: F401

__all__ = ["QEMError", "load"]
