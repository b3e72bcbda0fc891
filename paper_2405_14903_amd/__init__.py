"""MI355X-native differentiable MAC-grid Navier-Stokes step (NeuralFluid,
arXiv 2405.14903): HIP kernels for gfx950 behind a C ABI, with a thin PyTorch
binding, an autograd rollout with step checkpointing, and a continuously
batched serving loop.

The compute path is ``libneuralfluid.so`` (built in-tree by ``build.py``);
importing this package does not load it -- the first call does, and fails
loudly if it is missing.
"""
from .sim import (Sim, sim_create, sim_step, sim_project, sim_step_adjoint, poisson_solve,
                  sim_footprint, ellipsoid_poses, ellipsoid_poses_adjoint)

__all__ = ["Sim", "sim_create", "sim_step", "sim_project", "sim_step_adjoint", "poisson_solve",
           "sim_footprint", "ellipsoid_poses", "ellipsoid_poses_adjoint"]
