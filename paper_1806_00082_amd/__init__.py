"""MI355X-native hot path of the signed-particle Wigner Monte Carlo method with a
neural-network Wigner kernel (Sellier, Leygonie, Marceau Caron, arXiv:1806.00082).

Submodules:
  inputs   seeded synthetic workloads (meshes, potentials, eq.(6) bin counts)
  _lib     ctypes loader of libwigner.so (C ABI in include/wigner.h)
  ops      torch-facing argument marshalling for each C entry point
  sim      time loop driver (kernel rows -> tables -> sp_step -> sp_annihilate)
  learn    autograd Functions and the training loop of the learned kernel
  build    hipcc build of libwigner.so

Importing the package loads nothing; the HIP library is loaded on first use and its
absence is an error (there is no CPU fallback).
"""
__all__ = ["inputs", "ops", "sim", "learn", "build"]
