"""Writes the stored expected values under tests/golden/ (calls only the oracle and the input generators).

chain16_channels.txt: open-channel counts N_ch(E) of the random 16-orbital chain cell (seed 0) at the
64 energies linspace(-3, 3, 64), from the lead band structure (oracle.bands); a perfect crystal of
this cell must transmit exactly N_ch(E).  Run:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import bands  # noqa: E402


def main():
    cell = synth.chain_cell(16, 0)
    q = np.linspace(-np.pi, np.pi, 4096, endpoint=False)
    bb = bands.bloch_bands(*cell, q)
    lines = ["# E  N_ch  min|E_n(q)-E|   (chain_cell(16, seed=0), q-grid 4096)"]
    for E in np.linspace(-3.0, 3.0, 64):
        n, gap = bands.channel_count(*cell, E, bands=bb)
        lines.append(f"{E:.17g} {n} {gap:.3e}")
    with open(os.path.join(HERE, "chain16_channels.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
