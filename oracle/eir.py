"""Oracle of the transducer response (test infrastructure): every trace of a time-major
[M][L] array convolved in time with one causal kernel h (the measured signal is the
pressure convolved with the transducer's impulse response, Sec. 2.3), truncated to the
M samples, and its adjoint, the correlation with h.  FP64 NumPy; the convolution and
correlation of numpy are the definition written out.
"""
import numpy as np


def eir_apply(h, z):
    """out[m][l] = sum_k h[k] z[m-k][l], m = 0..M-1 (zero before the first sample)."""
    h = np.asarray(h, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    M = z.shape[0]
    return np.stack([np.convolve(z[:, l], h)[:M] for l in range(z.shape[1])], axis=1).reshape(z.shape)


def eir_adjoint(h, y):
    """out[m][l] = sum_k h[k] y[m+k][l] (zero past the last sample)."""
    h = np.asarray(h, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    M, nh = y.shape[0], h.size
    out = np.empty_like(y)
    for l in range(y.shape[1]):
        full = np.correlate(np.concatenate([y[:, l], np.zeros(nh - 1)]), h, mode="valid")
        out[:, l] = full[:M]
    return out
