"""Write the closed-form eigenvalue fixtures (calls only the oracle).

The values are the Dirichlet 7-point Laplacian's eigenvalues from the closed
form quoted in Section 4.1, at the grid sizes the tests and benchmarks use,
including the two accuracy test grids of Section 4.1 (200^3 and 200x201x202,
50 smallest).  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_form  # noqa: E402

CASES = [((16, 16, 16), 4), ((128, 128, 128), 16), ((256, 256, 256), 33), ((96, 96, 96), 8),
         ((464, 464, 464), 8), ((6, 7, 8), 12), ((200, 200, 200), 50), ((200, 201, 202), 50)]


def main():
    path = os.path.join(HERE, "laplace7_smallest.txt")
    with open(path, "w") as f:
        f.write("# Smallest eigenvalues of the Dirichlet 7-point Laplacian, closed form of Section 4.1.\n")
        f.write("# Written by tests/golden/make_golden.py from oracle.closed_form.\n")
        f.write("# nx ny nz index lambda i j k\n")
        for dims, m in CASES:
            lam, ijk = closed_form.smallest(*dims, m)
            for t in range(m):
                f.write("%d %d %d %d %.17g %d %d %d\n" % (*dims, t, lam[t], *ijk[t]))
    print(path)


if __name__ == "__main__":
    main()
