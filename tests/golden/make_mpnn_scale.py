"""Writes mpnn_c3_scale.txt: the energy scale s_E of the seeded random-init
message-passing target such that the RMS force component on the seeded
1536-atom triatomic liquid is 1 eV/Angstrom (fixed before any draft work).
Calls the FP64 oracle only."""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle.mpnn import MPNN  # noqa: E402
from paper_2606_02455_amd import workloads as W  # noqa: E402

WEIGHT_SEED = 17


def main():
    w = W.config("c3")
    net = MPNN(W.mpnn_weights(3, seed=WEIGHT_SEED), 3, rc=5.0, scale=1.0)
    t = time.time()
    E, F = net.energy_forces(w.species, w.positions, float(w.box[0]))
    rms = float(np.sqrt(np.mean(F ** 2)))
    with open(os.path.join(HERE, "mpnn_c3_scale.txt"), "w") as fh:
        fh.write("# s_E: RMS force component 1 eV/A on the seeded c3 configuration\n")
        fh.write(f"# weights: workloads.mpnn_weights(3, seed={WEIGHT_SEED}); oracle E(s=1) = {E!r}\n")
        fh.write(f"scale = {1.0 / rms!r}\n")
    print(f"rms force at s=1: {rms:.6g}; s_E = {1.0 / rms:.6g} ({time.time() - t:.1f} s)")


if __name__ == "__main__":
    main()
