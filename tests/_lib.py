"""Shared helpers of the test suite (no arithmetic of the method)."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_03964_amd", "libtfdp.so")


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2303_03964_amd.build import build_library
        build_library(verbose=False)
    return LIB


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def header_functions():
    """Function names declared in include/tfdp.h."""
    import re
    src = open(os.path.join(ROOT, "include", "tfdp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tfdp_[a-z_]+)\s*\(", src)))
