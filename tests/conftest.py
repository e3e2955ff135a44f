import os
import sys
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def load_golden(name):
    """Parse a tests/golden matrix file into {name: 2-D list of floats}."""
    out, cur = {}, None
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = []
            else:
                out[cur].append([float(t) for t in line.split()])
    return out


@pytest.fixture(scope="session")
def golden():
    return load_golden


class CountingAllocator:
    """An amg_allocator (device memory from torch's caching allocator) that
    counts live and peak bytes and the calls made, and can fail the k-th
    allocation (returns NULL) to force the library's out-of-memory path from
    the host."""

    def __init__(self, torch, fail_at=None):
        from paper_2007_00056_amd import hemamg

        self.live = self.peak = self.calls = 0
        self.sizes = {}
        self.fail_at = fail_at
        self.lock = threading.Lock()

        def alloc(n, stream):
            with self.lock:
                self.calls += 1
                if self.fail_at is not None and self.calls == self.fail_at:
                    return 0
            p = torch.cuda.caching_allocator_alloc(n, torch.cuda.current_device(), stream)
            with self.lock:
                self.sizes[p] = n
                self.live += n
                self.peak = max(self.peak, self.live)
            return p

        def free(p, stream):
            with self.lock:
                self.live -= self.sizes.pop(p)
            torch.cuda.caching_allocator_delete(p)

        self.impl = hemamg.Allocator(alloc, free)
        self.c = self.impl.c
