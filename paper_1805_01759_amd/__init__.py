"""MI355X (gfx950) solver for the complex L1-regularised least-squares problem
of super-resolving TomoSAR (Shi, Zhu, Yin, Bamler, arXiv 1805.01759).

The HIP library is loaded lazily by ``api``; ``synth`` (input generation) has
no dependency on it.
"""
__all__ = ["api", "synth"]
