"""FP64 CPU oracle for the facet-wise regularization step of Faceted HyperSARA.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library and
its Python binding) never does, and shares no code, table or helper with it.

Everything here is plain numpy / LAPACK in float64, written to be checked
against the paper by eye:

* ``filters``    -- Daubechies extremal-phase filters by spectral factorisation
                    (the eight wavelet bases of the SARA dictionary, Sec. 2.3.1).
* ``dwt``        -- zero-extended, expansive, multi-level separable 2D DWT and
                    its exact adjoint.
* ``sara``       -- the SARA dictionary Psi^dagger (8 Daubechies bases + Dirac,
                    divided by sqrt(9)), its adjoint Psi, and the explicit
                    faceted variant (Sec. 2.4.2, exact faceting).
* ``geometry``   -- tiles, overlapping facets, the triangular apodisation
                    window D_q, coefficient ownership (Sec. 2.4.2).
* ``prox``       -- the proximal operators of Table 1 (soft-threshold,
                    weighted SVT, l21 row shrink).
* ``step``       -- one facet step of Algorithm 2: the weighted nuclear-norm
                    dual update, the weighted l21 dual update and the gather
                    into the primal gradient (facet part of the aggregation);
                    its randomized form updates a random subset of facets.
* ``spectral``   -- the facet step with overlapping spectral facets (the
                    100-channel case read literally: contiguous blocks whose
                    low-rankness facets overlap by a few channels with a
                    triangular spectral ramp; a reading, not in the paper).
* ``nufft``      -- the measurement operator Phi = G F Z (Kaiser-Bessel
                    de-gridding on a 2x oversampled grid) and the data-fidelity
                    dual update with the preconditioned l2-ball projection by
                    forward-backward sub-iterations (Sec. 2.1, Alg. 2, Sec. 3.2).
* ``heuristics`` -- regularisation parameters (eqs. heuristic_fhs_sparsity and
                    heuristic_fhs_low_rank) and reweighting weights
                    (eqs. facet_hypersara_rank and facet_hypersara_sparsity).
"""
