"""Plain, slow FP64 CPU oracle of the displacement-based FFT solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or constant generators); the two meet
only at the seeded problem descriptions in ``workloads``.

Modules
-------
``dt``      Table 1 transforms (DFT, DCT-I, DST-I, DCT-III, DST-III), their
            inverses and the virtual-extension identities (Sec. 2.4, Tab. 1).
``fd``      HEX1 / TETRA2 finite-difference gradient and divergence with the
            symmetry / periodicity extensions (Sec. 2.5, Eqs. D1HG-D3HG,
            D1T1T2G-D3T1T2G, Remark 1, Eq. Continuous_der_symmetry_per).
``green``   Modified frequencies and the B0 / 2mu0 discrete Green operators
            (Eqs. modified_freq_hex1, freq_TETRA2, NSGO1_*, NSGO2_*).
``laws``    Constitutive laws: isotropic and rotated cubic elasticity, J2
            radial return with linear hardening, FCC crystal viscoplasticity.
``solver``  Algorithm 1 (algFFT): increments, fixed-point iterations,
            equilibrium criterion, Anderson acceleration on p, mixed control.

Parity status: every function is pinned by ``tests/test_oracle_*.py`` except
the Anderson iteration history (iteration counts and logs), which is
"parity unpinned" -- only the fixed point it converges to is pinned.
"""
