"""FP64 CPU oracle for generalized sampling with boundary-corrected Daubechies
scaling functions (Jacobsen, Nielsen, Rasmussen, "Generalized Sampling in
Julia", arXiv 1607.04091).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product library (``paper_1607_04091_amd``) never imports, links or executes
this package, and this package never imports the product library: the two
share no code, tables or constants.  The only shared module is the seeded
input generator ``workloads`` (no method arithmetic in it).

Every function is a plain, slow, obviously-correct restatement of the paper:

* ``daubechies``  -- filter taps h_k and the infinite product for phi-hat
                     (App. A, eq. for F[phi] as a product of m0).
* ``cdv``         -- Cohen-Daubechies-Vial boundary functions: their filters
                     (H, h) and the matrix dilation recursion for their
                     Fourier transforms (App. A.1).
* ``basis``       -- the change-of-basis matrix T of Sec. 4 (1D) and Sec. 5 /
                     App. C (2D tensor product), dense.
* ``ndft``        -- the NDFT and its adjoint by direct sums (Sec. 3.2).
* ``lsq``         -- the weighted least-squares solution (Sec. 2, Sec. 4.1)
                     by a library QR/SVD solver and by CGLS.
* ``cascade``     -- scaling functions in space on dyadic grids; used only to
                     pin the Fourier-side routines independently.
* ``cnn``         -- the learned warm start (not from the paper): 3x3
                     convolutions, the residual network, its loss, backward
                     pass and Adam, with optional bf16 storage rounding.
"""
