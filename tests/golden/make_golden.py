"""Writes the golden fixtures of this folder.  Calls only the oracle and the
seeded input generators; never the GPU library.

    python tests/golden/make_golden.py

The paper (arXiv:2110.13368) prints no field values, so these files are not
paper numbers: they freeze the oracle's output on tiny seeded cases so that an
accidental change to its arithmetic shows up, and they give the GPU tests a
fixed target.  Any change to them must name, in its commit message, the
reading of the paper that justifies it.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2110_13368_amd import workloads as W  # noqa: E402

CASES = {
    # name: (shape, n_sub, bc, n_cells, decay_mode, steps, seed)
    "tiny_mixed_once": ((6, 5, 4), 2, "mixed", 12, O.DECAY_ONCE, 4, 1),
    "tiny_mixed_thirds": ((6, 5, 4), 2, "mixed", 12, O.DECAY_THIRDS, 4, 1),
    "line_x_neumann_once": ((9, 1, 1), 1, "neumann", 3, O.DECAY_ONCE, 6, 2),
}


def case_spec(name):
    shape, n_sub, bc, n_cells, mode, steps, seed = CASES[name]
    rng = np.random.default_rng(W.SEED_BASE + 1000 + seed)
    spec = W.make_sim(rng, shape, (20.0, 15.0, 10.0), n_sub, dtype="f64", bc=bc, n_cells=n_cells,
                      cell_layout="uniform")
    if n_cells >= 2:
        spec.cells.pos[1] = spec.cells.pos[0]
    return spec, mode, steps


def run(name):
    spec, mode, steps = case_spec(name)
    sim = O.from_spec(spec, decay_mode=mode)
    sim.step(steps)
    return sim.get_field()


def main():
    for name in CASES:
        out = run(name)
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as f:
            f.write(f"# oracle field after the case's steps; shape {out.shape} (n_sub, nz, ny, nx)\n")
            f.write(f"# written by tests/golden/make_golden.py, case {name}: {CASES[name]}\n")
            for v in out.ravel():
                f.write(f"{v:.17g}\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
