"""The P2S network (Sec. 3.3): fully connected layers that map the per-pixel
high-order Zernike coefficients alpha_4..alpha_K to the M basis coefficients
beta, run independently at every pixel.

Readings (the layer sizes sit in a figure that is not available): layers are
y = W x + b with W [out][in]; ReLU after every layer but the last (beta may be
negative); the input is the raw coefficients in radians.

Parity: unpinned against the paper (the network's weights are random, not
trained); the oracle is the definition written out.
"""
import numpy as np


def forward(Ws, bs, x: np.ndarray) -> np.ndarray:
    """x [n_pix][in] -> [n_pix][out] in FP64."""
    h = np.asarray(x, dtype=np.float64)
    L = len(Ws)
    for l in range(L):
        h = h @ np.asarray(Ws[l], dtype=np.float64).T + np.asarray(bs[l], dtype=np.float64)
        if l < L - 1:
            h = np.maximum(h, 0.0)
    return h
