"""MI355X (gfx950) hot path of the P2S turbulence simulator.

``p2s``    -- ctypes binding of libp2s.so (the C ABI in include/p2s.h): fields,
              network, fused basis blur, tilt warp, whole frames.
``basis``  -- one-time host setup: PSF dataset and PCA basis (Sec. 3.2).
``build``  -- hipcc build of libp2s.so for gfx950.
"""
__all__ = ["p2s", "basis", "build"]
