"""Double-grid lattice-regularized DMC projection for AMD Instinct MI355X.

Hot path: hand-written HIP kernels for gfx950 in ``csrc/`` behind the C ABI of
``include/lrdmc.h`` (liblrdmc.so); ``lrdmc`` is the thin Python binding,
``inputs`` the seeded synthetic workloads, ``stats`` the estimator used by
the benchmark.  Method: Nakano, Maezono & Sorella, arXiv:1909.01589.
"""
__all__ = ["inputs", "lrdmc", "stats", "build"]
