"""Write linear_modes.json: eigenmodes of the linear-mode background.

Calls only the CPU oracle (its flux Jacobians). Run from the repository root:
    python -m problems.make_linear_modes
"""

import json
import os

import numpy as np

from oracle.modes import eigenmodes
from problems.modes import BACKGROUND, GAMMA, MODES_FILE, kkey


def main():
    table = {}
    for kvec in ((1, 1, 1), (1, 1, 0)):
        modes = eigenmodes(BACKGROUND, GAMMA, kvec)
        table[kkey(kvec)] = {
            name: dict(omega=om, R_re=[float(x) for x in np.real(R)],
                       R_im=[float(x) for x in np.imag(R)])
            for name, (om, R) in modes.items()}
    with open(MODES_FILE, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", os.path.relpath(MODES_FILE))


if __name__ == "__main__":
    main()
