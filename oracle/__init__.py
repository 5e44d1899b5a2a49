"""Plain FP64 CPU oracle of the HARP reduced-MBF array solver (arXiv 1702.03781).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here.
The GPU library never uses it, and it shares no code, header, table or constant
with the GPU library; the only common code is the seeded input generator in
``workloads/``, which contains none of the method's arithmetic.

Every function follows a passage of the paper and is written for a reader to
check against it by eye: no blocking, fusion or reordering beyond what the
definition states.  Library primitives (matrix products, QR, LAPACK solves) are
used as single steps.

Modules
-------
em        exact MBF reactions (Section II-A), far-field patterns (Eq. 1)
fit       HARP model construction (Eqs. 2-3, Section II-B)
fill      reduced-matrix fill from the model (Eq. 4)
solve     port excitations, dense LU solve, port admittances (Section I, II-C)
patterns  embedded element / array patterns (Eqs. 5-6)

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
except the physical fidelity of the synthetic elements (there is no antenna
mesh to compare with): that part is "parity unpinned".
"""
