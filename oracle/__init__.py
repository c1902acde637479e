"""FP64 CPU oracle for the PSE FTS mobility, its Brownian sampler and the
stresslet-constrained mid-point step (Fiore & Swan, "Rapid Sampling of
Stochastic Displacements in Brownian Dynamics Simulations with Stresslet
Constraints").

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  It shares no code with the HIP library and never imports it.

Everything is computed from the paper's definitions in plain FP64:

* conventions.py  -- 11-component force/velocity layout and the symmetric
                     traceless basis (Sec. II.B "Mobility relation for rigid
                     particles").
* pairfuncs.py    -- free-space and real-space pair mobilities (Eqs. MUF-MDC,
                     the Hasimoto splitting H(k,xi), Appendix A).
* ewald.py        -- dense real-space and wave-space parts of the grand
                     mobility (Eqs. MUFw-MDCw, pairsums) and their products.
* brownian.py     -- the split sampler (Eq. split, DFTsqrt): principal square
                     root of M_r and the wave-space noise map.
* integrator.py   -- the stresslet constraint (Eqs. rigidconstraint,
                     constrained_vel) and the mid-point scheme (Sec. III.D,
                     Appendix B).
* params.py       -- the quadrature error bound rule (Eq. bound, Table 1).

Functions whose result is not pinned by an independent check say
"parity unpinned" in their docstring.
"""
