"""MI355X (gfx950) refinement path of CppFlow (arXiv 2309.09102).

Submodules:
  cpf    binding of the HIP library libcpf.so (C ABI in include/cpf.h)
  synth  seeded synthetic workloads (robots, paths, candidate plans)
  build  hipcc build of libcpf.so

Importing the package does not load the HIP library; ``import
paper_2309_09102_amd.cpf`` does, and fails loudly if it is not built.
"""
__all__ = ["cpf", "synth", "build"]
