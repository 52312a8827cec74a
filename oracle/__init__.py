"""CPU oracle for the k-th eigenvalue of a symmetric H^2 matrix (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, header, table
or helper with the HIP library; both sides receive the same seeded inputs from
``paper_2311_08618_amd.workloads`` (which holds no arithmetic of the method).

Plain, slow and written for a reader holding the paper (Apriansyah & Yokota,
"Computing the k-th Eigenvalue of Symmetric H^2-Matrices"):

  * ``tree``    cluster tree, block tree (strong admissibility), colouring
                (Sec. 3.1 notation; Sec. 3.4 "any pattern of dense
                off-diagonal blocks").
  * ``build``   nested orthonormal shared bases, transfer matrices and
                couplings (Eqs. shared-bases and transfer-matrices, Sec. 3.1).
  * ``factor``  generalized H^2-LDL of A - sigma*I returning the inertia
                nu = #{lambda < sigma} (Secs. 3.2-3.4, Eq. inertia of Sec. 2,
                Sec. 4).
  * ``bisect``  slicing the spectrum (Algorithm 1) with inertia reuse (Sec. 4.2).
  * ``dense``   brute-force checkers: dense inertia, cyclic Jacobi eigensolver,
                closed-form 1-D Laplacian spectrum.

Pins (all in ``tests/test_oracle_pins.py``, marked "not gpu"):
  * the closed-form spectrum 2-2cos(j*pi/(n+1)) of the 1-D second-difference
    matrix, for every shift, through the full hierarchical path with and
    without fill-in, and through bisection at large n;
  * dense inertia of the assembled H^2 matrix and of the exact kernel matrix,
    k-th eigenvalues against LAPACK at loose and tight tolerance, and every
    eigenvalue of the circle matrix within half the paper's tolerance (Sec. 5.1);
  * the construction bound ||A - A~||_2 <= 10 eps ||A|| (n = 1024 and 8192),
    the row ID's Frobenius stopping rule and the block-row budget;
  * the tree: partition, depth and median split, the block tree tiling every
    entry once, a valid greedy colouring;
  * Sylvester/Haynsworth additivity after every level of the factorization;
  * the Jacobi eigensolver, the rank-revealing QR and Gershgorin bounds;
  * planted mistakes (a sampled far field, a dropped recompression, a wrong
    Schur sign, a transposed transfer matrix, a wrong admissibility test, a
    missing coupling) that one of the above must catch.
Individual factor values (pivots, ranks) depend on truncation: they are
"parity unpinned" one by one; their per-level sums are checked against the
bookkeeping of the factorization itself.
"""
