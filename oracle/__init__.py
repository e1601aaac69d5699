"""Plain FP64 CPU oracle for the D3Q19 MRT-Smagorinsky LES update.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in it.  The product (``paper_2512_23116_amd``) never touches it, and it
shares no code, header, table or constant generator with the HIP path.

Contents
--------
``d3q19``      velocity set, weights, moment matrix M and relaxation rates,
               transcribed from the paper's Appendix B (Fig. d3q19_table,
               eq. moment-matrix, eq. relaxation-matrix).
``ref_numpy``  the dense literal definition of one time step (eq. mrt_les_guo
               with eq. feq, eq. guo_force, eq. guo_velocity, eq. meq_fm,
               eq. yu_strain, eq. strain_norm, eq. les_viscosity), used for
               brute force on small lattices.
``ref_c``      the same definition as plain scalar C with OpenMP over z-planes
               (``ref_lbm.c``), loaded through ctypes; used for everything
               larger than brute-force sizes and timed as the CPU baseline.
``physics``    parameter relations of Sec. 2.1, 2.2, 3.1 and 4 (tau0 from Re,
               F0 from C_f, the K41 worked estimate).
``stats``      statistics of a per-cell field (two-pass, FP64), the
               shell-binned energy spectrum, structure functions, turbulence
               scales and isotropy (Sec. 2.2, 3.3, 5.3), the one-dimensional
               spectra and the spectral isotropy coefficient (App. spectral
               isotropy).

Every function cites the passage of the paper it follows.  Readings taken
where the paper is silent or inconsistent are stated where they are used.
Every function is pinned by tests/test_oracle_pins.py against closed forms,
invariants, printed values or brute force; the one comparison left unpinned
is pointwise agreement of long chaotic runs, which are compared through
statistics only.
"""
