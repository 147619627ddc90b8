"""MI355X-native fitness evaluation for elitist-mutated PSO velocity-model search.

Submodules:
  fd         problems, bilinear two-grid map, forward modelling, misfit and
             batched fitness (HIP library through the C ABI)
  pso        host FP64 particle swarm with elitist mutation
  surrogate  BF16 MFMA multilayer-perceptron surrogate and screening policy

Importing a submodule that needs the HIP library raises ImportError when
libempso.so has not been built; nothing falls back to a CPU path.
"""
__all__ = ["fd", "pso", "surrogate"]
