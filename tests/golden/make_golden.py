"""Write the stored oracle references for the full-size parity tests.

Calls only the CPU FP64 oracle (`oracle/`) and the seeded input generators
(`lc_inputs/`). Each reference is the field of one workload at a fixed set
of target cells, by direct periodic summation (route D: the convolution sum
of Eq. 11 summed over slices). Beside each array a JSON file records the
workload, the targets, the route, the digest of the exact inputs
(lc_inputs.sources_digest) and the SHA-256 of the oracle source it was
computed with.

    python tests/golden/make_golden.py [grid256] [grid512] [uneven]

grid256  256^3 x 40 slices: the 64^3 stride-4 sub-lattice (262,144 cells),
         dense kernel; also sum_c G_k(c) per slice (the kernel's DC value).
grid512  512^3 x 60 slices x 4 bands, Gaussian-field peak sources: the 16^3
         stride-32 sub-lattice per band, summed over the kernel's support.
uneven   the 16 uneven boxes with N > 128: the 16^3 stride-N/16 sub-lattice
         of each, dense kernel. (Boxes with N <= 128 are compared on the full
         grid against the naive-DFT route at test time.)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lc_inputs as li  # noqa: E402
import oracle  # noqa: E402


def oracle_sha() -> str:
    with open(os.path.join(ROOT, "oracle", "oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def save(name: str, arrays: dict, meta: dict):
    np.savez(os.path.join(HERE, name + ".npz"), **arrays)
    meta = dict(meta, oracle_c_sha256=oracle_sha(), threads=oracle.num_threads())
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"wrote {name}", flush=True)


def grid256():
    b = li.points_256c_40s().boxes[0]
    t0 = time.time()
    G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
    print(f"grid256 kernel {time.time() - t0:.0f} s", flush=True)
    tg = li.sublattice_cells(b.n, 4)
    J = np.zeros(len(tg))
    for i in range(0, len(tg), 16384):
        J[i:i + 16384] = oracle.field_direct(G, b.sources, tg[i:i + 16384])
        print(f"grid256 targets {i + 16384}/{len(tg)} {time.time() - t0:.0f} s", flush=True)
    gsum = G.sum(axis=(1, 2, 3))     # G^_k(0), for the mean of the field
    save("grid256_slices40_sublattice4", {"J": J, "gsum": gsum},
         {"workload": "lc_inputs.points_256c_40s()", "targets": "lc_inputs.sublattice_cells(256, 4)",
          "route": "D, dense kernel (oracle.build_G, oracle.field_direct)",
          "inputs_sha256": li.sources_digest(b)})


def grid512():
    t0 = time.time()
    b = li.bands_512c_60s(procs=8).boxes[0]
    print(f"grid512 sources {time.time() - t0:.0f} s", flush=True)
    tg = li.sublattice_cells(b.n, 32)
    J = oracle.field_direct_support(b.n, b.box, b.radii, b.supersample, b.bands, b.sources, tg)
    print(f"grid512 field {time.time() - t0:.0f} s", flush=True)
    save("grid512_slices60_bands4_sublattice32", {"J": J},
         {"workload": "lc_inputs.bands_512c_60s()", "targets": "lc_inputs.sublattice_cells(512, 32)",
          "route": "D over the kernel support (oracle.field_direct_support), all 4 bands",
          "inputs_sha256": li.sources_digest(b)})


def uneven():
    w = li.uneven_16boxes()
    arrays, meta = {}, {"workload": "lc_inputs.uneven_16boxes()", "route": "D, dense kernel",
                        "boxes": {}}
    for i, b in enumerate(w.boxes):
        if b.n <= 128:
            continue
        t0 = time.time()
        G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
        tg = li.sublattice_cells(b.n, b.n // 16)
        arrays[f"J{i}"] = oracle.field_direct(G, b.sources, tg)
        del G
        meta["boxes"][str(i)] = {"n": b.n, "slices": b.n_slices,
                                 "targets": f"lc_inputs.sublattice_cells({b.n}, {b.n // 16})",
                                 "inputs_sha256": li.sources_digest(b)}
        print(f"uneven box {i} N={b.n} K={b.n_slices} {time.time() - t0:.0f} s", flush=True)
    save("uneven16boxes_sublattice16", arrays, meta)


if __name__ == "__main__":
    which = sys.argv[1:] or ["uneven", "grid512", "grid256"]
    for w in which:
        {"grid256": grid256, "grid512": grid512, "uneven": uneven}[w]()
