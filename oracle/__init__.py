"""CPU oracle for the shape-gradient path (test infrastructure only).

Plain, slow, FP64 NumPy code that states what the GPU path must compute:

* ``sigma``      -- the five sigma_k building blocks (Appendix "Nonlinear
                    function definitions", Tab. nonlinearfunctions).
* ``lattice``    -- where each field component samples the material
                    (staggered Yee positions; a documented reading).
* ``primitives`` -- AutoDiffGeo primitives and their analytic partials
                    (Sec. "AutoDiffGeo", Tab. autodiffgeo).
* ``scene``      -- composition by eq:union / eq:intersection and the
                    difference of Sec. "Single-polarization blazed grating",
                    material scaling, the adjoint sensitivity of eq:1, the
                    reverse-mode gradient of eq:AD / eq:jaceps and central
                    finite differences of the same map.
* ``volavg``     -- the "Standard" volumetrically averaged permittivity of
                    Sec. "Approximating sub-pixel smoothing" (exact box
                    overlap, exact polygon clipping, supersampling).
* ``philox``     -- Philox4x32-10 counter-based normal generator (Salmon et
                    al., SC'11), for fields the GPU draws itself.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (closed forms, volumetric-averaging identities,
paper-printed values, brute force, FD-vs-analytic) except the sensitivity
constant c = -2i*omega of eq:1, which is pinned only through special cases
(see tests/test_oracle_gradient.py).
"""
