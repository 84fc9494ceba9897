"""FP64 CPU oracle for the P2S turbulence simulator (Mao, Chimitt & Chan,
"Accelerating Atmospheric Turbulence Simulation via Learned Phase-to-Space
Transform", ICCV 2021).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import it;
the product path never does.  It shares no code with the HIP kernels or their
host library: the only things both sides see are the seeded input arrays.

Each function follows the paper's steps in its own order and notation:

* ``zernike``  -- Zernike basis in Noll ordering (Sec. 2.2, Eq. 1).
* ``noll``     -- diagonal of the Noll covariance R_Z (Sec. 2.2).
* ``psf``      -- PSF formation from pupil phase (Sec. 2.2, Eq. 2).
* ``basis``    -- PSF dataset and PCA basis (Sec. 3.2).
* ``philox``   -- Philox4x32-10 counter-based generator + Box-Muller normals.
* ``fields``   -- spatially correlated Zernike fields by FFT filtering
                  (stands in for the anchor-grid draw of Sec. 3.4).
* ``mlp``      -- the P2S network applied per pixel (Sec. 3.3).
* ``blur``     -- spatially varying blur, exact (Eq. 3) and via the basis
                  (Eq. 4-5).
* ``warp``     -- tilt displacement by bilinear resampling (Sec. 2.2, 3.3).
* ``simulate`` -- one frame end to end (Fig. 3 pipeline, Sec. 3.5 colour).

Parity status of each function is listed in its module header.
"""
from . import zernike, noll, psf, basis, philox, fields, mlp, blur, warp, simulate  # noqa: F401
