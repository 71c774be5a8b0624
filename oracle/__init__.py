"""CPU FP64 oracle for Frequency-Splitting MLMC trace estimation.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library and its Python binding
never do, and it shares no code with them (only the seeded generators in
`synth` serve both).

Everything is float64 / complex128 numpy, written to be checked by eye against
the paper (Whyte, Stathopoulos, Romero, Orginos, "Optimizing Shift Selection in
Multilevel Monte Carlo for Disconnected Diagrams in Lattice QCD"):

* `lattice`  -- site indexing, gamma matrices, Gamma_n, the Wilson-Dirac
                operator (matrix-free and dense), Omega_p = W Pi_p
                (Introduction: the target Tr(Gamma Omega_p D^-1)).
* `clover`   -- the clover (Sheikholeslami-Wohlert) term of the improved
                Wilson operator named in the Results section: field strength
                from the four plaquette leaves, sigma_{mu nu} F_{mu nu} per site
                (a reading of conventions the paper does not print).
* `philox`   -- Philox4x64-10 counter RNG and the Z4 noise drawn from it
                (Introduction, eq. test: entries from {1,-1,i,-i}).
* `solver`   -- BiCGStab (van der Vorst 1992) for (D + sigma I) x = b
                (Sec. 3.1, eqs. shifted_linear_systems / conj_shifted_...).
* `fs`       -- exact level traces and variances on tiny lattices and the
                stochastic FS estimator with per-level mean and variance
                (Sec. 2.2-2.3, eqs. tele_sum_prod_disp, phi_prod, phi_single,
                fs_trace_est, practical_variance, total_var, tosv), and the
                variance-sampling phase with shared noise (Sec. 3.1).
* `probing`  -- displacement-p distance-k probing colourings and the FS
                estimator with full spin-colour dilution (Background,
                Probing; Sec. 3.1 and 3.4).
* `shifts`   -- shift selection: PCHIP interpolation of the sampled variances
                in log space, the iteration-count cost model and the argmin of
                the multilevel cost over the evaluation set (Sec. 3.2-3.3,
                eqs. ml_cost_shifts, opt_shifts).

Parity status of every function is recorded in its docstring: each is pinned
by a test that does not reuse the oracle's own formula (closed forms, exact
enumeration, symmetries, library routines).
"""
