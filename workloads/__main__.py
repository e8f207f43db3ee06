"""Regenerate the committed geometry files: python -m workloads [c2 c3 c4 c5_pool c3x8]."""
import sys
import time

from . import generate

for nm in sys.argv[1:] or ["c2", "c4", "c3", "c5_pool", "c3x8"]:
    t0 = time.time()
    g = generate(nm)
    print(nm, len(g["A"]), f"side={g['side']:.3f}", f"{time.time() - t0:.1f}s", flush=True)
