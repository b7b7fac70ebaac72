"""CPU oracle for the tight-focusing method (arXiv:2010.00409).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU definition of what the GPU library computes, in float64 numpy/scipy.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path and never
imports it; the product path never routes through it.

Modules
-------
``dft``      direct per-axis DFT with exact integer phases (small grids)
``psatd``    the vacuum spectral step, Sec. II.A, Eqs. (3)-(4)
``pulse``    pulse on the focusing sphere and mapping into the periodic
             layer, Sec. II.B Eqs. (5)-(11), Sec. II.C Eqs. (12)-(13),
             Sec. III.B.1 (Gaussian beam)
``mapping``  cut-out of the primary pulse, Sec. II.C Eqs. (14)-(16)
``fno``      Fourier neural operator forward/backward (parity unpinned by
             the paper; pinned by finite differences)

Readings taken where the paper is silent or garbled are stated in each
module's docstring.
"""
