"""Writes poisson_spectra.txt from the closed form (no oracle call needed)."""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def extremes(dims, N):
    lo = 4.0 * math.sin(math.pi / (2 * (N + 1))) ** 2
    hi = 4.0 * math.sin(N * math.pi / (2 * (N + 1))) ** 2
    return dims * lo, dims * hi


def main():
    path = os.path.join(HERE, "poisson_spectra.txt")
    head = [ln for ln in open(path) if ln.startswith("#")]
    rows = []
    for name, dims, N in [("poisson2d", 2, 32), ("poisson2d", 2, 8), ("poisson3d", 3, 128),
                          ("poisson3d", 3, 16)]:
        lo, hi = extremes(dims, N)
        rows.append(f"{name} {dims} {N} {lo!r} {hi!r}\n")
    with open(path, "w") as f:
        f.writelines(head + rows)


if __name__ == "__main__":
    main()
