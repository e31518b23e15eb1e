"""Impulse-response record of the oracle and its spectrum peaks (section
Validation, Table 2).  TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

The spectrum analysis is written independently of the GPU package's modal
helper: a Hann-windowed FFT zero-padded eight times, the maximum of the
power spectrum in a window around each expected frequency, refined by the
vertex of the parabola through the power of its bin and its two
neighbours.
"""
import numpy as np


def record(sim, cell, comp, n_samples, every):
    """Displacement component comp (0, 1, 2) of cell ``cell`` of the oracle
    Sim after every ``every`` steps, n_samples values."""
    out = np.empty(int(n_samples))
    for i in range(int(n_samples)):
        sim.step(int(every))
        out[i] = sim.read_state()["u"][cell, comp]
    return out


def spectrum_peaks(x, dt, guesses, rel_window=0.2, pad=8):
    """Frequency (Hz) of the power-spectrum maximum of the sampled signal x
    (sample spacing dt) within a relative window around each guess."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    w = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n) / (n - 1))
    P = np.abs(np.fft.rfft((x - x.mean()) * w, n=pad * n)) ** 2
    df = 1.0 / (pad * n * dt)
    f = []
    for g in guesses:
        lo = max(1, int(g * (1 - rel_window) / df))
        hi = min(P.size - 2, int(g * (1 + rel_window) / df) + 1)
        i = lo + int(np.argmax(P[lo:hi + 1]))
        y0, y1, y2 = P[i - 1], P[i], P[i + 1]
        den = y0 - 2 * y1 + y2
        f.append((i + (0.5 * (y0 - y2) / den if den != 0 else 0.0)) * df)
    return f
