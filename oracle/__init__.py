"""Plain FP64 CPU oracle of fast FCM (Su & Keaveny, arXiv 2310.12651).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP implementation (no kernels, headers, helpers, tables or constants); the two
meet only at the seeded inputs produced by ``workloads.py``.

Modules
-------
closed_forms  pair-mobility closed forms S, Q, T, R, K, P (Sec. 2.2, Sec. 3.2,
              Sec. 3.4), the fast-FCM correction blocks (eqs. correction_VF,
              correction_WF, correction_WT) and the self corrections (App. B).
fastfcm       the fast-FCM algorithm of Sec. 4: hashing, sorting/cell lists,
              spreading with the modified kernel, the Fourier Stokes solve,
              interpolation and the pairwise correction.
lattice       the exact periodic FCM mobility written as a Fourier lattice
              sum (App. A made periodic) -- the plain definition that fast FCM
              approximates to a tolerance.
derive        committed derivations of stored parameters (cut-off radii).

Every function names the passage of the paper it follows.  Where the paper
is garbled or silent, the reading taken is stated at the point of use.
"""
