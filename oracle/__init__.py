"""CPU FP64 oracle for the kernel-free boundary integral (KFBI) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It is a plain, slow, numpy/scipy implementation written
from the paper (Zhou, Li, Ying, "A Cartesian grid-based boundary integral method for
moving interface problems") and shares no code with the HIP path.

Modules
-------
spectral  Fourier differentiation / integration / Hilbert transform (Sec. 5.3 remark).
geometry  markers, grid-line crossings, inside/outside labels, irregular arms (Sec. 4.2).
kfbi      jumps (App. A.1), corrected RHS (Sec. 4.2.1), DST-I solve, box data (Sec. 4.1),
          corrected interpolation (Sec. 4.3) -> one operator apply.
gmres     restarted GMRES with modified Gram-Schmidt (Sec. 4 intro, matrix-free).
thetal    theta-L / small-scale-decomposition Hele-Shaw step (Sec. 3.1, 5.1-5.3).
stokes    modified Stokes interface problem on the MAC grid: App. A.2 jumps, corrected
          scheme (Sec. 4.2.2), velocity traces, double-layer operator of eq. ms-bie.
convnet   FP64 1-D convolutional warm-start network forward/backward (reference for
          gradient checks of the learned warm start; not part of the paper).

Parity status of every function is listed in its module header ("pinned by ...").
"""
