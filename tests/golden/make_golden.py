"""Writes the exact-rational golden fixtures in this folder.

Calls only ``oracle.exact`` (Fraction arithmetic, no rounding).  The paper
prints no worked Poisson example, so these fixtures pin the floating-point
oracle to the exact discrete solution of tiny problems instead: the bordered
Neumann system of the staggered 7-point operator (paper, "Fluid Mechanics"
subsection; Neumann walls and a fixed reference value for the pressure
correction, boundary-condition paragraph after eq. ``pressure``).

Run:  python tests/golden/make_golden.py
"""
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact import exact_bordered_solve  # noqa: E402

CASES = {
    # name: (nx, ny, nz, Lx, Lz, y faces)
    "exact_4x3x2": (4, 3, 2, Fraction(4), Fraction(2),
                    [Fraction(-1), Fraction(-1, 2), Fraction(1, 4), Fraction(1)]),
    "exact_3x4x3": (3, 4, 3, Fraction(3, 2), Fraction(5, 2),
                    [Fraction(-1), Fraction(-3, 4), Fraction(0), Fraction(1, 3), Fraction(1)]),
    "exact_2x2x1": (2, 2, 1, Fraction(1), Fraction(7, 3),
                    [Fraction(0), Fraction(1, 5), Fraction(2)]),
}


def rhs(nx, ny, nz):
    """Deterministic small-integer right-hand side (not mean-free on purpose,
    so the removed weighted mean is pinned too)."""
    return [[[Fraction(((7 * i + 3 * k + 5 * j * j + i * k) % 11) - 4)
              for i in range(nx)] for k in range(nz)] for j in range(ny)]


def main():
    for name, (nx, ny, nz, Lx, Lz, yf) in CASES.items():
        f = rhs(nx, ny, nz)
        phi, mu = exact_bordered_solve(f, Lx, Lz, yf)
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as fh:
            fh.write("# exact rational solution of the bordered staggered Neumann problem\n")
            fh.write("# written by tests/golden/make_golden.py (oracle.exact only)\n")
            fh.write(f"shape {ny} {nz} {nx}\n")
            fh.write(f"Lx {Lx}\nLz {Lz}\n")
            fh.write("yf " + " ".join(str(y) for y in yf) + "\n")
            fh.write(f"mu {mu}\n")
            for j in range(ny):
                for k in range(nz):
                    for i in range(nx):
                        fh.write(f"{j} {k} {i} {f[j][k][i]} {phi[j][k][i]}\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
