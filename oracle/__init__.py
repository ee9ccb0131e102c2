"""Plain, slow FP64 CPU oracle for the FFT-accelerated BIE hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table
or constant generator with the HIP library under ``paper_2608_16208_amd/``
and imports nothing from it.

Reference: W. Hua, J. Lai, H. Li, W. Lu, "An FFT-accelerated boundary integral
equation method for wave scattering by smooth surfaces in three dimensions".

Where the method approximates a quantity that has a plain definition (the
azimuthal Fourier coefficients of rho^-1 and of e^{ik rho}/rho, eq. (3.9) and
the definition of <f>_m in Sec. 3.2; the singular-factor coefficients A_m(b),
eq. (3.26)), the oracle evaluates that definition directly with heavily
oversampled, graded composite Gauss-Legendre quadrature.  Nothing here uses
the Newton root, the smooth-factor FFT, Miller's recurrence or the FFT
convolutions of Sec. 3.3: those are what the GPU path must reproduce.

Modules
-------
geometry  star-family surfaces r(t, theta) and the cancellation-free
          difference r(v) - r(u) of Remark 4.2 (line integral in parameter space)
coeffs    direct-quadrature <rho^-1>_l and <e^{ik rho}/rho>_n (Sec. 3.2)
special   A_m(b) from its defining integral, eq. (3.26)
banded    the O(M) route of Sec. 3.2.1: <rho^2>_n, the m0 rule of eq. (3.13)
          and the banded system of eqs. (3.14)-(3.18), solved densely
"""
