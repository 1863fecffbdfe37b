"""Writes the shape terms N_zz - N_xx of the film grids that
paper_2603_03706_amd/workloads.py stores (FILM_SHAPE_TERMS).

The film workload's bias puts the uniform mode of the out-of-plane
magnetised block at 5 GHz: B0 = 2 pi 5 GHz / gamma + mu0 Ms (N_zz - N_xx),
with N the volume-averaged demagnetizing tensor of the block (the average of
the cell-pair Newell tensor over all cell pairs), which for a rectangular
block is Aharoni's closed form.  Calls only the oracle.

    python tests/golden/film_shape_terms.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import theory  # noqa: E402

SHAPES = [(128, 128, 32), (16, 12, 4), (16, 16, 4), (8, 6, 3), (6, 5, 3), (6, 5, 2), (5, 4, 2)]


def shape_terms():
    out = {}
    for nx, ny, nz in SHAPES:
        n_xx, _, n_zz = theory.prism_demag_factors(float(nx), float(ny), float(nz))
        out[(nx, ny, nz)] = float(n_zz - n_xx)
    return out


if __name__ == "__main__":
    print("FILM_SHAPE_TERMS = {")
    for k, v in shape_terms().items():
        print(f"    {k}: {v!r},")
    print("}")
