"""CPU oracle for the block-Jacobi sweeping preconditioner (arXiv 2209.10886).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (``paper_2209_10886_amd`` and its HIP library) never imports it, and
this package imports nothing from the product path: the two share no code.  The
only common module is ``workload`` (seeded input generators, no solver
arithmetic).

Plain, slow and obviously correct: numpy / scipy in complex128, one Python loop
per subdomain, scipy's SuperLU for every sparse solve.  Each function cites the
passage of the paper it follows (section / equation / definition / table).

Modules
-------
layout     multi-indices, the lexicographic orders, the pair map m, groups (Sec. 2)
fd         5-point discretisation with the Robin face closure (Sec. 3, eq. (1))
dd         local problems, lifting, scattering operator, (I - S) g = b (Secs. 3-4)
sweep      SGS sweeping preconditioner and block-Jacobi partial sweeps (Secs. 5-6)
krylov     restarted right-preconditioned GMRES / FGMRES (Sec. 7)
gradient   adjoint-state gradient of a data misfit w.r.t. m = 1/c^2
"""
