"""Writes the stored exact determinants under tests/golden/.

Calls only the CPU oracle (its C Bareiss, oracle/bareiss.c) and the seeded
input generators; no value here comes from the GPU library.  The n = 1024
case takes tens of minutes on 8 cores.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    # random dense n = 1024, entries uniform in [0, 255], the plain headline workload
    "dense_n1024_u0_255_seed1024": dict(n=1024, lo=0, hi=255, seed=1024),
    # random dense n = 512, entries uniform in [-128, 127] (largest batched size)
    "dense_n512_s128_seed3": dict(n=512, lo=-128, hi=127, seed=3),
}


def main(names):
    for name in names or CASES:
        c = CASES[name]
        A = synth.dense_uniform(c["n"], c["lo"], c["hi"], c["seed"])
        t0 = time.time()
        d = oracle.det_bareiss_c(A)
        rec = dict(c, generator="synth.dense_uniform", oracle="oracle.det_bareiss_c",
                   det_hex=hex(d), det_bits=abs(d).bit_length(),
                   seconds=round(time.time() - t0, 1))
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json"), "w") as f:
            json.dump(rec, f, indent=1)
        print(name, rec["det_bits"], "bits", rec["seconds"], "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
