"""MI355X-native (gfx950) truncated-Fock statevector engine for CV-ADAPT-VQE.

The compute path lives in libfock.so (hand-written HIP kernels behind a C ABI,
declared in include/fock.h); this package only binds it (lib), wraps the
adjoint energy gradient as a torch.autograd.Function (autograd), drives the
learned warm start (warmstart) and the benchmarks (kbench, sweep_bench), and
builds the library (build).
"""
from . import lib  # noqa: F401

__all__ = ["lib"]
