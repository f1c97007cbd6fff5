"""FP64 CPU oracle for the ET-AIM marching hot path (Kaur & Yilmaz, 1408.7060).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library; the only common input is the seeded geometry/random arrays
of the ``workloads`` module.

Plain, slow, obviously correct numpy/scipy in float64/complex128:

* ``physics``     constants and the pulse / time-step / history-depth rules
                  (Sec. 2.2, 2.3, Sec. 3 eq. (3)-(4), Table I)
* ``cppif``       causal piecewise-polynomial interpolatory temporal basis
* ``quadrature``  triangle rules (7-point degree-5 rule, exact collapsed
                  Gauss-Legendre product rule, simplex monomial formula)
* ``geometry``    triangle and RWG geometry
* ``potentials``  closed-form static potentials of a flat triangle
* ``kernels``     envelope Green-function kernels of the differentiated EFIE
* ``zfill``       envelope impedance matrices Z_m (eq. (4)) and the
                  frequency-domain EFIE matrix at f_c
* ``excitation``  incident envelope (eq. (1)) and excitation vectors V_l
* ``march``       direct ET-MOT march of eq. (4) and the ET-AIM march of eq. (5)
* ``aim``         auxiliary grid, moment-matching projection, grid Green
                  functions, near zone, pre-correction, AIM matvec (Sec. 4)
* ``farfield``    scattered far-field envelopes and the energy objective
* ``adjoint``     adjoint (backward) march and gradient
* ``mie``         Mie series of a PEC sphere and the dB-error norm eq. (2)

Parity status of each function is stated in its docstring; anything not
pinned by an independent check says "parity unpinned".
"""
