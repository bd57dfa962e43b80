"""Write tests/golden/workload_stats.json: exact nonzero counts of A per workload.

Calls only the oracle (FP64 Siddon traversal) and the seeded geometry
description in synth.  The benchmark reads the stored numbers for its
algorithmic-traffic model; tests check a small case against brute force.

Usage: python tests/golden/make_workload_stats.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "workload_stats.json")


def main(names):
    stats = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        gd = synth.geometry(name)
        g = oracle.Geometry.from_dict(gd)
        t = time.time()
        nnz, hits = oracle.count_nnz(g)
        n_rays = len(g.angles) * g.nu * g.nv
        stats[name] = dict(nnz=nnz, hit_rays=hits, rays=n_rays, voxels=g.nx * g.ny * g.nz,
                           voxel_views=g.nx * g.ny * g.nz * len(g.angles),
                           segments_per_hit_ray=nnz / max(hits, 1), nnz_per_voxel_view=nnz / (g.nx * g.ny * g.nz * len(g.angles)))
        print(name, stats[name], f"{time.time() - t:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(stats, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cgls32", "medical256"])
