"""Device floors for the roofline: python -m paper_1812_06160_amd.calibrate [bytes]

Prints one JSON object from ilu_calibrate: stream-read and copy GB/s, the
published-value hop latency (one XCD, across XCDs) and the kernel launch cost.
"""
import ctypes as C
import json
import sys

import numpy as np

from . import _lib as L


def calibrate(nbytes: int = 0) -> dict:
    lib = L.load()
    out = np.zeros(5, np.float64)
    L.check(lib.ilu_calibrate(int(nbytes), out.ctypes.data_as(C.c_void_p), 5), "ilu_calibrate")
    return dict(read_gbs=round(out[0], 1), copy_gbs=round(out[1], 1), hop_ns_same_xcd=round(out[2], 1),
                hop_ns_cross_xcd=round(out[3], 1), launch_us=round(out[4], 3))


if __name__ == "__main__":
    print(json.dumps(calibrate(int(sys.argv[1]) if len(sys.argv) > 1 else 0)))
