"""Write c2_workload.json: oracle figures of the 1,000,000-Gaussian 1256x828
workload (seed 1002) that the benchmark's roofline uses as algorithmic work.

pairs: sum over pixels of the Gaussians whose compact box holds the pixel, in
depth order up to the pixel's stop point (the (pixel, Gaussian) pairs the
compositing of Eq. (rendering) evaluates); tile_pairs: (tile, Gaussian) keys
of 16x16 tiles.  Calls only the oracle."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_06876_amd import synth  # noqa: E402


def main():
    scene, cam, _ = synth.c2_inputs()
    pr = oracle.project(scene, cam)
    r = oracle.render_rows(pr)
    keys, _, _ = oracle.bin_tiles(pr, 16, 16)
    out = dict(workload="1,000,000 clustered Gaussians SH3, 1256x828, seed 1002",
               pairs=int(r["pairs"].sum()), pairs_per_pixel=float(r["pairs"].mean()), tile_pairs=int(len(keys)),
               visible_gaussians=int(pr.valid.sum()), flagged_pixels=int(r["flag"].sum()),
               contributors=int(r["ncontrib"].sum()))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_workload.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
