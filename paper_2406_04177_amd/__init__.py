"""MI355X (gfx950) implementation of the voxel-graph diffusion-transformation
method of Klai, Monga, Jouini and Pot (arXiv:2406.04177).

The simulation runs in hand-written HIP kernels behind the C ABI of
``include/vgsim.h`` (``libvgsim.so``); this package is its Python binding:

    Graph.from_masks(masks)          pore-voxel graph (Sec. II.A)
    Simulation(graph, params, ...)   explicit / implicit steps, mass totals
    autograd.simulate_totals(...)    differentiable total curves (adjoint)

``inputs`` holds the seeded synthetic workloads.
"""
from .inputs import ModelParams, POOL_NAMES  # noqa: F401

__all__ = ["Graph", "Simulation", "ModelParams", "POOL_NAMES"]


def __getattr__(name):
    if name == "Graph":
        from .graph import Graph
        return Graph
    if name == "Simulation":
        from .sim import Simulation
        return Simulation
    raise AttributeError(name)
