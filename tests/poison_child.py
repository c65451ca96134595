"""Child process of test_gpu_poison.py: runs the solves listed there with
the library's NaN poisoning of new floating-point device buffers
(SPFAS_POISON=1, set by the parent) and saves the states."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np  # noqa: E402

from test_gpu_poison import run_all  # noqa: E402

if __name__ == "__main__":
    out = sys.argv[1]
    for name, (p, s, it) in run_all().items():
        np.save(os.path.join(out, f"{name}_p.npy"), p)
        np.save(os.path.join(out, f"{name}_s.npy"), s)
    print("child done", flush=True)
