"""CPU reference ("oracle") for the particle-relaxation step of the
feature-preserving particle generation method (FPPG, arXiv 2501.03056, section 3.3).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, brute-force FP64
restatement of what one relaxation iteration computes. It exists to check the
GPU library against. Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the GPU path never calls it and
shares no code with it (the only common dependency is the seeded input
generator package `synth`, which holds none of the method's arithmetic).

Modules (each function cites the passage it follows):
  kernel     Wendland C2 kernel, Eq. 16-17, and the pair-force coefficient of Eq. 15
  cells      cell keys and the canonical (cell, id) order of the rebuilt cell list
  neighbors  the binary32 neighbour predicate, brute force over all pairs
  force      relaxation acceleration (Eq. 15) with the particle-class interaction rule
  geometry   facet planes, barycentric coordinates, closest point, winding number
  step       time step, velocity reset, displacement, tangential projection (Eq. 22-25)
             and the projection / revert rules of section 3.3.3
  hvp        Jacobian of the force field (Hessian-vector product of the pair energy)
  metrics    force residual and density-uniformity loss
  csg        Boolean assemblies: part signed distances, boundary membership
  local      the same step at full size (candidate searches, pinned to brute force)
  register   facet subdivision and registration on a grid, Morton code and
             compact hash of the registered cells (sections 3.1.1, 3.1.3)
  multires   per-particle resolution levels with the pair length of Eq. 6

The front-end modules generate, features and band are imported by name.

Readings of points where the paper is silent or garbled are listed where they
are used; the functions with no independent pin say "parity unpinned" in their
docstring (time-step rule, feature-line motion, volume revert rule, metrics).
"""
from . import kernel, cells, neighbors, force, geometry, step, hvp, metrics, csg, local, register, multires  # noqa: F401
