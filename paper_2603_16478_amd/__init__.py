"""MI355X (gfx950) implementation of the per-time-step analytical adjoint of
"Fast and Reliable Gradients for Deformables Across Frictional Contact
Regimes" (arXiv 2603.16478): a C-ABI HIP library (include/adjoint.h) and its
Python binding.  Nothing is loaded at import time; ``native.load()`` loads the
built library and raises if it is missing."""

__all__ = ["native", "build"]
