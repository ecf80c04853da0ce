"""Writes the regression fixtures in this folder from the oracle only."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenes import city_scene, open_plane_2k  # noqa: E402


def lloyd_case():
    sc = open_plane_2k(eps="rule")
    sc.gamma = np.array([0.8 * np.exp(1j * np.pi / 8)])
    idx = np.arange(0, 4096, 256) + 37
    return sc, idx


def city_case():
    sc = city_scene(n_blocks=3, n_rays=600, grid=3, freqs=(300.0, 800.0), max_refl=4, city_seed=7, panels=2,
                    complex_gamma=True)
    return sc, np.arange(len(sc.rcv))


CASES = {"open_plane_2k_lloyd.json": lloyd_case, "city_small.json": city_case}


def main():
    oracle.build(force=False)
    for name, fn in CASES.items():
        sc, idx = fn()
        P, TL = oracle.forward(sc.table, sc.gamma, sc.rcv[idx], sc.freqs, sc.eps, c=sc.c, gate=sc.gate)
        out = {"receivers": idx.tolist(), "P_re": P.real.tolist(), "P_im": P.imag.tolist(), "TL": TL.tolist()}
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", name)


if __name__ == "__main__":
    main()
