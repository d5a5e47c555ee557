"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import numpy as np
import torch

# Tolerance of the FP64 path against the FP64 oracle, per element:
# |gpu - oracle| <= RTOL * (|oracle| + max|oracle| over the instance).
# The natural ends are exactly 0 and interior second derivatives span several
# orders of magnitude, so a pure relative bound would be ill-posed near zero.
RTOL = 1e-10


def close(g, o, rtol=RTOL):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    if o.size == 0:
        return True, 0.0
    scale = np.max(np.abs(o))
    err = np.abs(g - o)
    ok = bool(np.all(err <= rtol * (np.abs(o) + scale)))
    return ok, float(np.max(err / (np.abs(o) + scale + 1e-300)))


def assert_close(g, o, what="", rtol=RTOL):
    ok, worst = close(g, o, rtol)
    assert ok, "%s: worst scaled error %.3e > %.1e" % (what, worst, rtol)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()
