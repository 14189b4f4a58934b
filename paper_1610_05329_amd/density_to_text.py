"""Convert a binary density file written by dgpe_write_density to text.

The file holds Nx*Ny*Nz float64 values, row-major [x][y][z] with x slowest and
no header; each output line is "x y z density" with x_i = (i - Nx/2) dx.

    python -m paper_1610_05329_amd.density_to_text FILE NX NY NZ DX DY DZ > out.txt
"""
import sys

import numpy as np


def main(argv):
    if len(argv) != 8:
        print(__doc__, file=sys.stderr)
        return 2
    path = argv[1]
    n = tuple(int(v) for v in argv[2:5])
    d = tuple(float(v) for v in argv[5:8])
    dens = np.fromfile(path, dtype="<f8")
    if dens.size != n[0] * n[1] * n[2]:
        print(f"{path}: {dens.size} values, expected {n[0] * n[1] * n[2]}", file=sys.stderr)
        return 1
    dens = dens.reshape(n)
    axes = [(np.arange(n[a]) - n[a] // 2) * d[a] for a in range(3)]
    out = sys.stdout
    for i in range(n[0]):
        for j in range(n[1]):
            for k in range(n[2]):
                out.write(f"{axes[0][i]:.6f} {axes[1][j]:.6f} {axes[2][k]:.6f} {dens[i, j, k]:.17e}\n")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
