"""Seeded workload generator for the BDDC hot path.

This package turns the paper's model problem (Sec. 2-3: the divergence-free
virtual element discretization of 3D Stokes on a cube mesh) into the data the
hot path consumes: per-subdomain reduced saddle-point matrices, right-hand
sides, the global interface numbering and the per-entity primal constraint
functionals (Sec. 4.1-4.2 and the primal recipe of Sec. 5.1).

It holds no BDDC, Schur-complement, scaling, coarse-space or Krylov
arithmetic: both the CPU oracle and the HIP library consume its output as
plain data.  Its own correctness is pinned by the tests (DoF counts of the
paper's tables, patch test, divergence-free discrete velocity, h-rates).
"""
