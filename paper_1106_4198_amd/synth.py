"""Seeded synthetic power spectrograms for online IS-NMF.

Stand-in for the audio of the paper's experiments (section 3: power
spectrograms of single-channel tracks, 512-sample windows), which are not
available.  The generator follows the IS-NMF generative model: a frame is a
nonnegative mixture of K spectra times multiplicative exponential noise,

    V = max( (W_true H_true) * E , 1e-12 ),
    W_true ~ Gamma(shape 0.5, scale 1)   (F x K)
    H_true ~ Gamma(shape 0.3, scale 1)   (K x N)
    E      ~ Exponential(1)              (F x N)

and the starting dictionary W0 ~ Uniform(0.5, 1.5).  Only random draws are
made here; no step of the factorization method is computed.

Reproducibility: numpy PCG64 streams keyed by SeedSequence(seed,
spawn_key=...).  Frames are drawn in fixed chunks of CHUNK columns with one
key per chunk, so a prefix of a stream is the same whatever total length is
requested.  Arrays are Fortran-ordered float32 (column n of V is frame n,
contiguous in memory).
"""
from __future__ import annotations

import numpy as np

CHUNK = 4096
FLOOR = 1e-12


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed), spawn_key=tuple(key))))


def true_dictionary(F: int, K: int, seed: int) -> np.ndarray:
    """W_true ~ Gamma(0.5, 1), F x K, float64."""
    return np.asfortranarray(_rng(seed, 0).gamma(0.5, 1.0, size=(K, F)).T)


def initial_dictionary(F: int, K: int, seed: int) -> np.ndarray:
    """W0 ~ Uniform(0.5, 1.5), F x K, float32 (Fortran order)."""
    return np.asfortranarray(_rng(seed, 1).uniform(0.5, 1.5, size=(K, F)).T.astype(np.float32))


def _chunk(Wt: np.ndarray, F: int, K: int, seed: int, c: int):
    g = _rng(seed, 2, c)
    Ht = g.gamma(0.3, 1.0, size=(CHUNK, K)).T       # K x CHUNK
    E = g.exponential(1.0, size=(CHUNK, F)).T        # F x CHUNK
    return Ht, E


def frames(F: int, K: int, N: int, seed: int, start: int = 0, with_h: bool = False,
           threads: int = 0):
    """Frames [start, start+N) of stream `seed`: float32 F x N (Fortran).

    With with_h, also returns the float64 H_true columns used (K x N).
    threads > 1 draws the chunks in parallel (same values)."""
    Wt = true_dictionary(F, K, seed)
    out = np.empty((F, N), dtype=np.float32, order="F")
    hs = np.empty((K, N), dtype=np.float64, order="F") if with_h else None
    c0 = start // CHUNK
    c1 = (start + N + CHUNK - 1) // CHUNK

    def fill(c):
        Ht, E = _chunk(Wt, F, K, seed, c)
        lo = max(start - c * CHUNK, 0)
        hi = min(start + N - c * CHUNK, CHUNK)
        pos = c * CHUNK + lo - start
        blk = (Wt @ Ht[:, lo:hi]) * E[:, lo:hi]
        np.maximum(blk, FLOOR, out=blk)
        out[:, pos:pos + hi - lo] = blk
        if with_h:
            hs[:, pos:pos + hi - lo] = Ht[:, lo:hi]

    if threads > 1 and c1 - c0 > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(c0, c1)))
    else:
        for c in range(c0, c1):
            fill(c)
    if with_h:
        return out, hs
    return out


def problem(F: int, K: int, N: int, seed: int):
    """(V float32 F x N, W0 float32 F x K) for one stream."""
    return frames(F, K, N, seed), initial_dictionary(F, K, seed)
