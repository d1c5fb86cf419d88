"""MI355X-native HSE screened Fock-like exchange (Sato, Taniguchi, Shinohara, Yabana, Sec. II C).

Submodules:
  synth    -- seeded synthetic inputs (lattice, k-mesh, orbitals)
  _native  -- ctypes binding of libfockmi.so
  api      -- Plan: apply / energy / vjp / taylor_step / orthonormalize / apply_batched
  autograd -- torch.autograd.Function wrappers over the Plan
  build    -- hipcc build of libfockmi.so

Importing the package does not load the library; `api` and `autograd` do.
"""

__all__ = ["synth", "api", "autograd", "build"]
