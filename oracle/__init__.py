"""Plain FP64 CPU oracle of the Galilean-PSATD particle-in-cell step.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call anything in this package.  The HIP path in
``paper_1608_00215_amd`` never imports it, and it imports nothing from there:
the two share no kernels, helpers, tables or constants.  The only module both
sides use is ``workload`` (seeded synthetic inputs, none of the method's
arithmetic).

Everything here is written from Kirchen et al., "Stable discrete
representation of relativistically drifting plasmas" (arXiv:1608.00215):

* ``spectral``     -- wavevectors, the forward/inverse FFT (numpy), the modes
                      held at zero, and the Galilean-PSATD field update
                      (update equations for B and E, paper's main display).
* ``coefficients`` -- C, S, nu, theta and chi_1..chi_3 of that display,
                      evaluated through their Duhamel integrals (see module
                      docstring for why, and for the pins).
* ``particles``    -- B-spline shapes, deposition, gather, Galilean position
                      advance and the relativistic Boris momentum push
                      (transformed equations of motion).
* ``pic``          -- one full step in the order the paper states it.
* ``diagnostics``  -- field energy, Gauss and continuity residuals.

Normalised units throughout: c = eps0 = m_e = e = 1 unless passed explicitly.
Every floating-point quantity is float64.
"""

from . import coefficients, diagnostics, particles, pic, spectral  # noqa: F401
