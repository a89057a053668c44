"""Compute the PNA degree normaliser delta for each synthetic workload.

delta = mean over every node of ln(d + 1), d the in-degree, over 10,000 graphs
of the synthetic generator drawn with seed 3000 + c.  It calls only the seeded
generator and the oracle's CSR, and prints the constants that the workload
presets carry.
"""
import numpy as np

from paper_2207_11333_amd.synth import make_batch
from oracle.pna import csr_build

SHAPES = {0: (5, 30, 0), 1: (10, 60, 1), 3: (10, 70, 1)}


def main():
    for c, (lo, hi, fe) in SHAPES.items():
        b = make_batch(3000 + c, 10000, lo, hi, fe)
        csr = csr_build(b.graph_ptr, b.edge_index, b.num_nodes)
        delta = float(np.mean(np.log(csr.deg.astype(np.float64) + 1.0)))
        print(f"DELTA_C{c} = {delta!r}")


if __name__ == "__main__":
    main()
