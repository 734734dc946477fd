"""Write workload0_oracle.txt: FP64 oracle values of the workload-0 frame
(10,000 Gaussians, 64x48) at a seeded sample of pixels. Calls only the
oracle and the seeded input generators; the test that reads the file pins
the oracle against unintended changes of its arithmetic.

    python tests/golden/make_workload0_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import scenegen  # noqa: E402


def sample_pixels():
    rng = np.random.default_rng(20261202)
    return sorted({(int(i), int(j)) for i, j in zip(rng.integers(0, 64, 96),
                                                     rng.integers(0, 48, 96))})


def main():
    sc = scenegen.make_scene(0)
    cams = scenegen.make_cameras(0)
    ref = oracle.render(sc, cams["poses"][0], cams["intrinsics"][0], 64, 48)
    lines = ["# FP64 oracle, workload 0 (cube10k_sh0_64x48), one camera at (0, 0, -5)",
             "# written by tests/golden/make_workload0_oracle.py (oracle only)",
             "# counters: " + " ".join(f"{k}={v}" for k, v in ref.counters.items()),
             "# i j r g b depth alpha"]
    for i, j in sample_pixels():
        r, g, b = ref.rgb[j, i]
        lines.append(f"{i} {j} {r:.17g} {g:.17g} {b:.17g} {ref.depth[j, i]:.17g} "
                     f"{ref.alpha[j, i]:.17g}")
    with open(os.path.join(HERE, "workload0_oracle.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
