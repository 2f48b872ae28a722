"""Plain FP64 CPU oracle of the implicit APIC MPM step with spatially varying surface
energy (Chen et al., arXiv 2101.12408).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py may import or run anything in this package.  The GPU library never
calls it and shares no code with it; the two meet only at the seeded scene generators
in mpm_scenes (which hold none of the method's arithmetic).

Every function works on dense natural-order numpy float64 arrays: node (i_0,...,i_{d-1})
of the n^d cell-centred grid has linear index i_0 + n*(i_1 + n*i_2) and position
(i + 1/2) dx.  The modules follow the paper's section order:

  bspline   quadratic B-spline weights at cell-centred nodes        (Section 4.2)
  sampler   union-of-spheres level set, marching triangles/tets,
            per-triangle surface samples                           (Section 4.1.1)
  resample  nearest parents, balance particles, mass split          (Sections 4.1.2-4.1.3)
  transfer  P2G, grid set-up, G2P with merge                        (Sections 4.2, 5)
  energy    e(y), its gradient (eq. fe) and Hessian-vector product  (Section 4.3.1)
  solve     Newton-CG momentum solve, implicit heat solve           (Sections 4.3.1-4.3.2)
  step      one full time step                                      (Section 4 list of steps)

Where the paper leaves a point open, the function's docstring states the reading it takes.
"""
from . import bspline, sampler, resample, transfer, energy, solve, step  # noqa: F401
