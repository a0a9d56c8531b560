"""FP64 CPU oracle for the rank-adaptive sweep-based SI-DSA (Guo & Peng, arXiv 2603.25233).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_2603_25233_amd``) may import, link or execute anything in this package.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: the only module both
sides read is ``workloads`` (seeded synthetic inputs, no method arithmetic).

Every function follows a passage of the paper and says which one.  It is plain
and slow on purpose: numpy/scipy in float64, plus one small plain-C transport
sweep (``csweep.c``) so that grids of 256x256 cells stay affordable.

Modules
-------
quadrature   Chebyshev-Legendre CL(N_theta, N_z) rule (Appendix A).
dg           Upwind DG-Q1 discretisation on a Cartesian mesh (Sec. 2.1, Appendix B):
             cell matrices from the weak form by Gauss quadrature, sparse assembly.
sweep        Transport sweep, forward and transposed (Sec. 2.2, "Transport sweeps").
dsa          Diffusion correction (Sec. 2.2, eq. (DSA)); MIP discretisation, direct solve.
si           Full-rank SI-DSA (Sec. 2.2).
lowrank      Low-rank SI-DSA (Alg. 1) with MGS2-A (Alg. 2), greedy random sampling
             (Sec. 3.2), inner stopping (Sec. 3.3) and the single truncation.
adjoint      Discrete adjoint of the coupled S_N-DG system, detector functional and
             cross-section gradients.
metrics      Compression ratio, oversampling, effective rank (Sec. 4).
"""
