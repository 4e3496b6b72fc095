"""Writes the closed-form fixtures in this folder (uses only the math module).

ones_n*.txt: singular values of the n x n bidiagonal with d = e = 1.  B^T B is
tridiagonal with diagonal (1, 2, ..., 2) and off-diagonal 1, whose eigenvalues
are 4 cos^2(k pi / (2n + 1)), k = 1..n, so sigma_k = 2 cos(k pi / (2n + 1)),
descending in k.
"""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    for n in (1, 2, 5, 40, 100):
        path = os.path.join(HERE, f"ones_n{n}.txt")
        with open(path, "w") as f:
            f.write(f"# sigma_k = 2 cos(k pi / (2n+1)), n = {n}, d = e = 1\n")
            for k in range(1, n + 1):
                f.write(repr(2.0 * math.cos(k * math.pi / (2 * n + 1))) + "\n")


def deflation_cases():
    """The paper's N = 3 deflation examples (Section 4.2.1, after eq.
    M-condition), instantiated with values whose rotations are exact-ish.
    tol = 8 * 2^-52 * max(max d, max|z|) = 2^-50 for all four (max = 0.5).

    Each case: sorted d (d_1 = 0), z, then the expected d, z and status
    (0 survivor, 1 small z, 2 d close to d_1, 3 close pair) from the paper's
    formulas: r = sqrt(z_a^2 + z_b^2), the zeroed entry 0.
    """
    t = 2.0 ** -50
    cases = []
    # (1) |z_1| < tol: z_1 set to tol
    cases.append(("small_z1", [0.0, 0.25, 0.5], [2.0 ** -70, 0.5, 0.25],
                  [0.0, 0.25, 0.5], [t, 0.5, 0.25], [0, 0, 0]))
    # (2) |z_3| < tol: z_3 set to 0
    cases.append(("small_z3", [0.0, 0.25, 0.5], [0.5, 0.25, 2.0 ** -70],
                  [0.0, 0.25, 0.5], [0.5, 0.25, 0.0], [0, 0, 1]))
    # (3) |d_1 - d_i| < tol: r = sqrt(z_1^2 + z_i^2), d_i = 0, z_i = 0
    r = math.sqrt(0.375 * 0.375 + 0.5 * 0.5)
    cases.append(("d_close_to_zero", [0.0, 2.0 ** -60, 0.5], [0.375, 0.5, 0.25],
                  [0.0, 0.0, 0.5], [r, 0.0, 0.25], [0, 2, 0]))
    # (4) |d_i - d_j| < tol, i = 3, j = 2: z_j = r, z_i = 0, d_j replaced by d_i
    r = math.sqrt(0.375 * 0.375 + 0.5 * 0.5)
    d3 = 0.5 - 2.0 ** -54
    cases.append(("close_pair", [0.0, 0.5 - 2.0 ** -53, d3], [0.25, 0.375, 0.5],
                  [0.0, d3, d3], [0.25, r, 0.0], [0, 0, 3]))
    path = os.path.join(HERE, "deflation_n3.txt")
    with open(path, "w") as f:
        f.write("# Paper Section 4.2.1, the N = 3 deflation examples (four cases)\n")
        f.write("# name | d | z | expected d | expected z | expected status\n")
        for name, d, z, ed, ez, st in cases:
            f.write(" | ".join([name, " ".join(map(repr, d)), " ".join(map(repr, z)),
                                " ".join(map(repr, ed)), " ".join(map(repr, ez)),
                                " ".join(map(str, st))]) + "\n")


if __name__ == "__main__":
    main()
    deflation_cases()
