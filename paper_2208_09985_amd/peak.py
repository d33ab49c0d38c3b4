"""ctypes binding of libscrooge_peak.so: the resource microbenchmarks that
state the roofline's measured peak (32-bit bitwise VALU issue, LDS bandwidth,
load latencies, shader clock).  Argument marshalling only.

    python -m paper_2208_09985_amd.peak      # one JSON line
"""
from __future__ import annotations

import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscrooge_peak.so")


class PeakResult(ctypes.Structure):
    _fields_ = [
        ("valu_lane_ops_per_s", ctypes.c_double),
        ("valu_t64_ops_per_s", ctypes.c_double),
        ("lone_issue_cycles", ctypes.c_double),
        ("lone_dep_cycles", ctypes.c_double),
        ("lone_dpp_cycles", ctypes.c_double),
        ("lds_bytes_per_s", ctypes.c_double),
        ("lds_lat_cycles", ctypes.c_double),
        ("l2_lat_cycles", ctypes.c_double),
        ("sclk_mhz", ctypes.c_double),
        ("valu_kernel_ms", ctypes.c_double),
        ("num_cu", ctypes.c_int32),
        ("valu_waves", ctypes.c_int32),
    ]


def measure(device: int = 0) -> dict:
    """Run the microbenchmarks on `device`; returns the figures as a dict."""
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_09985_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.scg_peak_measure.argtypes = [ctypes.c_int, ctypes.POINTER(PeakResult)]
    lib.scg_peak_measure.restype = ctypes.c_int
    r = PeakResult()
    rc = lib.scg_peak_measure(device, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"scg_peak_measure failed ({rc})")
    return {name: getattr(r, name) for name, _ in PeakResult._fields_}


if __name__ == "__main__":
    import torch  # noqa: F401  (initialises the HIP runtime the same way the benchmark does)
    print(json.dumps(measure(0)), flush=True)
