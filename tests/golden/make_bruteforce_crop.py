"""Writes bruteforce_1024_crop.npz: the brute-force fluence of Eq. 1-3 (FP64 ray
march, 4096 directions per pixel) on the 128x128 crop rows 448..575, columns
448..575 of the 1024x1024 benchmark scene, and the FP64 oracle's HRC fluence on
the same crop (the method's own approximation error, for reference).  Calls
only the oracle and the seeded scene generator.

    python tests/golden/make_bruteforce_crop.py      (a few minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bruteforce  # noqa: E402
from oracle import hrc as oracle  # noqa: E402
from scenes import config3  # noqa: E402

CROP = (448, 576, 448, 576)
M = 4096


def main():
    sc = config3()
    bf = bruteforce.fluence(sc.eps, sc.sigma, M=M, crop=CROP)
    F = oracle.fluence(sc.eps, sc.sigma)
    r0, r1, c0, c1 = CROP
    np.savez_compressed(os.path.join(HERE, "bruteforce_1024_crop.npz"), crop=np.array(CROP),
                        directions=np.array(M), bruteforce=bf,
                        oracle_hrc=F[r0:r1, c0:c1])
    rmse = float(np.sqrt(np.mean((F[r0:r1, c0:c1] - bf) ** 2)))
    print(f"oracle HRC vs brute force on the crop: RMSE {rmse:.4g}, "
          f"mean brute-force fluence {bf.mean():.4g}")


if __name__ == "__main__":
    main()
