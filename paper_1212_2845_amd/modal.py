"""Impulse response and modal spectrum of a lattice (the paper's dynamic
validation: section Validation, Table 2, and the beam frequencies of the
equation given there).

``record`` steps a simulation on its GPU stream and samples one state word
of one cell every ``every`` steps into a device buffer (``vx_probe``), with
a single host synchronisation at the end.  ``peaks`` returns the
frequencies of the strongest local maxima of the Hann-windowed amplitude
spectrum, each refined by the vertex of the parabola through the
log-magnitudes of its bin and the two neighbours.  ``beam_frequencies`` is
the Euler-Bernoulli cantilever formula with the standard mode constants.
"""
import numpy as np

# Roots k_n L of 1 + cos(kL) cosh(kL) = 0 (clamped-free beam): the mode
# constants K_n = (k_n L)^2 of the paper's beam formula.
_KL = [1.8751040687, 4.6940911330, 7.8547574382, 10.9955407349, 14.1371683910, 17.2787595320]


def beam_frequencies(E, I, mass_per_length, L, n=6):
    """Natural frequencies (Hz) of a clamped-free Euler-Bernoulli beam,
    omega_n = K_n sqrt(E I / (m L^4))."""
    return [(kl * kl) * np.sqrt(E * I / (mass_per_length * L ** 4)) / (2 * np.pi) for kl in _KL[:n]]


def record(sim, cell, word, n_samples, every):
    """Run n_samples * every steps of ``sim`` and return word ``word`` (an
    index into paper_1212_2845_amd.WORDS) of cell ``cell`` after every
    ``every`` steps, as float64 numpy values."""
    import torch
    from . import WORDS
    if isinstance(word, str):
        word = WORDS.index(word)
    sim.bind()
    dev = sim._ws.device
    cells = torch.tensor([int(cell)], dtype=torch.int32, device=dev)
    out = torch.empty(int(n_samples), dtype=torch.float64 if sim.precision == 64 else torch.float32, device=dev)
    # the probe and the steps run on the handle's stream; the tensors were
    # made on torch's current stream, which must finish first
    torch.cuda.synchronize(dev)
    for i in range(int(n_samples)):
        sim.step_enqueue(int(every))
        sim.probe(cells, word, out[i:i + 1])
    sim.status()
    return out.cpu().numpy().astype(np.float64)


def peaks(signal, dt_sample, n_peaks, floor=1e-9, contrast=10.0, halfwidth=64):
    """Frequencies (Hz, ascending) of the n_peaks strongest resonances in the
    amplitude spectrum of ``signal`` (mean removed, Hann window): local
    maxima above ``floor`` times the largest that stand ``contrast`` times
    above the median of the spectrum within ``halfwidth`` bins (a resonance
    is a few bins wide; the smooth leakage of the record's start and end
    has shallow maxima of no such contrast)."""
    x = np.asarray(signal, dtype=np.float64)
    x = (x - x.mean()) * np.hanning(x.size)
    Z = np.abs(np.fft.rfft(x))
    df = 1.0 / (x.size * dt_sample)
    top = Z.max()
    idx = [i for i in range(1, Z.size - 1)
           if Z[i] > Z[i - 1] and Z[i] >= Z[i + 1] and Z[i] > floor * top
           and Z[i] >= contrast * np.median(Z[max(0, i - halfwidth):i + halfwidth + 1])]
    idx = sorted(idx, key=lambda i: -Z[i])[:n_peaks]
    out = []
    for i in sorted(idx):
        a, b, c = np.log(Z[i - 1]), np.log(Z[i]), np.log(Z[i + 1])
        den = a - 2 * b + c
        d = 0.5 * (a - c) / den if den != 0 else 0.0
        out.append((i + d) * df)
    return out
