"""Plain FP64 CPU oracle for improved W-stacking (Ye, Gull, Tan & Nikolic 2021).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library.

Modules
-------
kernel_design  least-misfit gridding function C and correction h
               (Sec. 3.3, eqs. csum2 and norm_bound).
plan           normalised coordinates, n0, n_scale and the w-layer range
               (Sec. 5.1, 5.3, eqs. n_params, N_{w'}+W).
wstack         Algorithm 5 (dirty map by 3-D gridding) and Algorithm 6
               (model visibilities by 3-D degridding), step by step.
dft            the exact direct Fourier transform pair the method
               approximates (Sec. 2, eq. fourier_visibility; Sec. 5.2).

Everything is float64 / complex128 and written for clarity, not speed.
"""
