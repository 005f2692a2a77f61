import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_example1():
    """Parse tests/golden/example1.txt (Section 4, Example 1)."""
    A = np.zeros((4, 3, 3))
    P = np.zeros((4, 3, 3))
    alpha = None
    iters = {}
    with open(os.path.join(ROOT, "tests", "golden", "example1.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "A":
                A[:, int(t[1]), int(t[2])] = [float(v) for v in t[3:7]]
            elif t[0] == "PINV":
                P[:, int(t[1]), int(t[2])] = [float(v) for v in t[3:7]]
            elif t[0] == "ALPHA":
                alpha = float(t[1])
            elif t[0] == "ITERS":
                iters[t[1]] = int(t[2])
    return A, P, alpha, iters


@pytest.fixture(scope="session")
def example1():
    return load_example1()


# ------------------------------------------------------------------ GPU helpers (used by -m gpu tests)
@pytest.fixture(scope="session")
def qctx():
    import paper_2605_01464_amd as q

    ctx = q.Context(0)
    yield ctx
    ctx.close()


def to_dev(A, dtype="f32"):
    """numpy (4, m, n) float64 -> contiguous device tensor of float32/float64 (the values both sides see)."""
    import torch

    t = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float32 if dtype == "f32" else torch.float64)
    return t.cuda()


def to_np(t):
    return t.detach().cpu().double().numpy()


def rel_fro(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))
