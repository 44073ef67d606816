"""Recycled shifted solver for MI355X (gfx950, FP64).

Solves the shifted systems (A + gamma_l E_k) x = b of Kilmer & de Sturler's
subspace-recycling method with hand-written HIP kernels behind the C ABI in
``include/rsr.h``.  Submodules:

  * ``rsr``      -- ctypes binding of the C ABI (device memory from torch);
  * ``irn``      -- outer edge-preserving iteration driving the solver;
  * ``autograd`` -- ``RecycledShiftSolve`` with the adjoint backward;
  * ``synth``    -- seeded synthetic inputs (phantoms, PSFs, noise, shifts);
  * ``build``    -- hipcc build of ``librsr.so``.

Nothing is imported eagerly, so ``synth`` can be used without the library.
"""
__all__ = ["rsr", "irn", "autograd", "synth", "build"]
