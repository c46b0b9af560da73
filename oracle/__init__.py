"""FP64 CPU oracle for algebraic hybridization of the H(div) problem on RT_k
hexahedra (Dobrev, Kolev, Lee, Tomov, Vassilevski, arXiv:1801.08914).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library
(``paper_1801_08914_amd``) never imports, links or calls anything here, and
nothing here imports the GPU library: the two share no code, tables or
constant generators.  Inputs come from the neutral ``synth`` module.

It is a plain, slow, obviously correct restatement of what the method computes:

* ``rt_basis``     RT_k reference basis on [0,1]^3 (nodal, closed/open points)
* ``quadrature``   tensor Gauss-Legendre rules
* ``geometry``     trilinear map, Jacobian
* ``element``      local matrix M_T and load f_T of the form
                   (alpha u, v) + (beta div u, div v) = (f, v)   (Sec. 3.2)
* ``topology``     faces, owners, orientation codes, multiplier ids, CSR pattern
* ``hybrid``       local Schur complements H_T = C_T M_T^{-1} C_T^T, global H,
                   r = C A^{-1} f, recovery of the broken solution (Thm 2.1)
* ``conforming``   the plain definition: P, A = P^T A_hat P, direct solve
* ``mixed``        the hybridized mixed form H~ (Sec. 3.2), an independent
                   route to H
* ``pcg``          Jacobi-preconditioned CG on H lam = r (Sec. 6.1 stopping rule)

Letters: this code calls the mass coefficient ``alpha`` and the div-div
coefficient ``beta``; the paper's weak form uses the opposite letters
(beta for the mass term, alpha for div-div, Sec. 3.2 eq. (weak_hdiv)).

Parity pins for each function live in ``tests/test_oracle_*.py``.
"""
