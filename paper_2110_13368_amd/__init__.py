"""voxlod: MI355X-native LOD diffusion-decay step with cell sources.

Importing the package loads nothing; the HIP library is loaded on first use by
``paper_2110_13368_amd.binding`` and a missing or unloadable library raises.
"""
__all__ = ["autograd", "binding", "workloads"]
