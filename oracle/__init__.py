"""FP64 CPU oracle for the multi-beam CCM eigenvalue RFI flagger.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
restatement of the method of Bai et al., "Radio frequency interference
identification using eigenvalue decomposition for multi-beam observations"
(arXiv 2512.16278). Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_2512_16278_amd``) never imports, calls or links anything here, and
nothing here imports the product path: the two share no code. Inputs are
plain NumPy arrays; the seeded input generator lives in its own module and is
not imported here either.

Modules (each function cites the passage of the paper it follows):

* ``ccm``      -- exact per-cell sums and the Pearson correlation matrix
                  (Sec. 3.2, Eq. 1).
* ``eig``      -- eigendecomposition and the normalised dominant-eigenvalue
                  statistic (Sec. 3.3, Eq. 2), by LAPACK and by an own cyclic
                  Jacobi.
* ``clip``     -- iterative one-sided Gaussian clipping of the statistic into
                  the combined mask (Sec. 3.3, Sec. 4.5 eigenvalue threshold),
                  batch and pooled-stream forms.
* ``bandpass`` -- ArPLS bandpass (Sec. 3.1) and the non-centred CCM of the
                  bandpass-subtracted power (the raw second-moment reading).
* ``eigvec``   -- per-beam eigenvector threshold (Sec. 3.3 last paragraph,
                  Sec. 4.5 eigenvector threshold).
* ``pipeline`` -- the whole per-block path composed from the above.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, worked examples, brute force and library special cases.
No function is "parity unpinned" except the agreement of the masks with the
paper's own FAST masks, which cannot be checked (no data; Sec. 2).
"""
