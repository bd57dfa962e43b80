"""The oracle: a plain, slow, FP64 CPU implementation of the Krylov CBCT path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything here.  The GPU library (``paper_2211_14212_amd``) never imports it,
and this package never imports the GPU library: the two share no code.  The
only code both sides use is the seeded input generator package ``synth``,
which holds none of the method's arithmetic.

Contents
  projector.py  FP64 Siddon forward projection A x and its scatter adjoint
                A^T y (C, OpenMP; ``siddon.c``), paper Sec. 1 eq. (original_pbm).
  dense.py      brute-force dense A for tiny grids, closed-form box and
                sphere chords (NumPy).
  interp.py     the unmatched, voxel-driven interpolating back projector B that
                GPU toolboxes use in place of A^T (NumPy), Sec. 2.1.4.
  solvers.py    CGLS, LSQR, LSMR (all with Tikhonov damping), hybrid LSQR
                with lambda fixed or chosen by GCV / the discrepancy principle,
                AB- and BA-GMRES, isotropic TV and IRN-TV with inner CGLS
                (NumPy).

Pins (``tests/test_oracle_*.py``, all CPU-only) tie each function to
something other than itself: closed-form chords, brute force on tiny grids,
the adjoint identity, the Krylov-subspace optimality that defines each solver
(checked against an explicitly orthonormalised Krylov basis), SciPy's
independent LSQR/LSMR, dense normal-equation solves, and hand-derived values
in ``tests/golden/``.  No function here is "parity unpinned".
"""
from .projector import (Geometry, adjoint, build, count_nnz, forward, forward_rays, num_threads, ray_segments,
                        set_num_threads)
from . import dense, interp, solvers

__all__ = ["Geometry", "forward", "adjoint", "forward_rays", "ray_segments", "count_nnz", "num_threads",
           "set_num_threads", "build", "dense", "interp", "solvers"]
