"""Writes oracle/tables/weights_d{d}_R{R}_ell5.npz: the oracle's reconstruction
vectors for every (dimension, radius) pair, solved in 50-digit arithmetic and
rounded once to float64.  Calls only oracle.weights.

    python -m oracle.build_tables
"""
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import weights  # noqa: E402

if __name__ == "__main__":
    for d, R in [(2, 2), (2, 3), (3, 2), (3, 3)]:
        fname = os.path.join(weights._CACHE_DIR, f"weights_d{d}_R{R}_ell{weights.ELL_HAT}.npz")
        if os.path.exists(fname):
            os.remove(fname)
        t = time.time()
        weights.tables(d, R)
        print(f"d={d} R={R}: {time.time() - t:.1f} s", flush=True)
