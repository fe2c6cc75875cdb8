"""Writes realistic_board_probes.npz: the FP64 oracle's full run of the
444 x 364 x 60 realistic board (20000 steps, 16 probes), for the GPU's
full-run parity test.  Calls only the oracle and the input generator.

Stored: every 4th sample of each probe series (the pulse's highest frequencies
span well over 100 steps, so nothing is lost for an L2 comparison), and the
spectral peaks of the full-resolution series (rectangular window, zero padding
to 2^15, peaks above 1 % of the maximum and above 0.5 GHz).

    python tests/golden/make_realistic_probes.py [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import boardgen  # noqa: E402
import oracle  # noqa: E402

DECIMATE = 4


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    b = boardgen.realistic_board()
    t0 = time.time()
    r = oracle.run(b, threads=threads)
    n_fft = oracle.default_nfft(b.steps)
    f = oracle.bin_freqs(n_fft, r.dt)
    peaks = []
    for p in range(len(b.probes)):
        X = np.abs(oracle.probe_fft(r.probes[p], n_fft))
        peaks.append(oracle.find_peaks(X, f, f_min=0.5e9))
    npk = max(len(x) for x in peaks)
    pk = np.full((len(peaks), npk), np.nan)
    for p, x in enumerate(peaks):
        pk[p, :len(x)] = x
    out = os.path.join(HERE, "realistic_board_probes.npz")
    np.savez_compressed(out, series=r.probes[:, ::DECIMATE], decimate=DECIMATE, steps=b.steps,
                        dt=r.dt, peaks_hz=pk, n_fft=n_fft)
    print(f"{out}: {len(b.probes)} probes x {b.steps} steps in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
