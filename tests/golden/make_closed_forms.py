"""Writes closed_forms.txt: textbook heat-equation series (no oracle call)."""
import os

import numpy as np


def S(a, t, terms=4001):
    k = np.arange(1, terms, 2)
    return float(np.sum(4.0 / (k * np.pi) * np.sin(k * np.pi * a) * np.exp(-k * k * np.pi ** 2 * t)))


def P0(a, t, terms=4001):
    k = np.arange(1, terms)
    return float((1.0 - a) - np.sum(2.0 / (k * np.pi) * np.sin(k * np.pi * a) * np.exp(-k * k * np.pi ** 2 * t)))


def D(t):
    return float(np.exp(-2.0 * np.pi ** 2 * t))


VALUES = {
    "S(0.5,0.05)^2": lambda: S(0.5, 0.05) ** 2,
    "S(0.5,0.05)*S(0.25,0.05)": lambda: S(0.5, 0.05) * S(0.25, 0.05),
    "P0(0.5,0.05)": lambda: P0(0.5, 0.05),
    "P0(0.1,0.05)": lambda: P0(0.1, 0.05),
    "P0(0.1,0.01)": lambda: P0(0.1, 0.01),
    "D(0.05)": lambda: D(0.05),
    "D(0.01)": lambda: D(0.01),
}

if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "closed_forms.txt")
    header = [ln for ln in open(path).read().splitlines() if ln.startswith("#")]
    with open(path, "w") as f:
        f.write("\n".join(header) + "\n")
        for name, fn in VALUES.items():
            f.write("%-26s %.12f\n" % (name, fn()))
