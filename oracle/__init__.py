"""FP64 CPU oracle for the w-stacking w-projection measurement operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code, tables or constants with the
HIP library; the two meet only through the seeded input generators in
``paper_1903_06555_amd.synthetic`` (which hold none of the method's
arithmetic).

Every routine is plain, slow FP64 numpy/scipy written from the paper
(Pratley, Johnston-Hollitt & McEwen 2019, "w-stacking w-projection hybrid
algorithm for wide-field interferometric imaging: implementation details and
improvements"):

- ``dft``       direct evaluation of the measurement equation, Eq. (1);
- ``taper``     the radial Kaiser-Bessel anti-aliasing pair g / k used in
                Eqs. (4) and (6), and the separable textbook pair;
- ``wkernel``   the radial (Hankel) w-projection kernel of Eq. (6), the
                support rule and the tap geometry of Eq. (5);
- ``operator``  Phi_k = W_k GC_k F Z S~_k (Eqs. (2)-(5)) and the stacked
                adjoint of Eq. (7);
- ``stacking``  conjugate-symmetry folding (Eq. (8)) and the k-means
                w-stacking of Algorithm 1.

Parity status of each function is listed in its module header.
"""
