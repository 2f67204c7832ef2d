"""Plain FP64 CPU oracle of the PDF solver's per-iteration hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The GPU library shares no code with it: no kernels, headers, helpers, tables or
pre/post-processing.  The only shared module is ``seeded_inputs`` (random
draws, profile geometry), which holds none of the method's arithmetic.

Everything here is NumPy/SciPy in float64 / complex128, written from the
paper's equations (Sec. 2-3, Eqs. 1-19) with library primitives (FFT, matmul,
LU, Bessel functions) as single steps and no blocking or fusion.

Modules
  operators   domain / receiver Green's operators and the incident field (Sec. 2.1)
  fourier     truncated Fourier basis synthesis and analysis (Sec. 2.3)
  forward     method-of-moments forward solve, Mie series, noise (Sec. 2.1, 4.2)
  loss        composite loss, hand adjoint gradient (Sec. 3.2, Eqs. 13-19)
  init        back-propagation start and the single-step alpha_0 (Sec. 3.1, Eq. 12)
  cco         contrast-compensated operator and image error (Sec. 2.4, Eqs. 10-11)
  adam        Adam update (Sec. 3.3)
  solver      one reconstruction: init, Adam iterations, image (Sec. 3, Fig. 3)

Functions whose result the paper does not fix are flagged in their docstring;
every other function is pinned by tests under ``tests/`` against closed
forms, library routines, brute force or invariants.
"""
