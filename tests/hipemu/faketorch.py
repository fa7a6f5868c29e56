"""A numpy stand-in for the few torch calls that bench.py, __graft_entry__.smoke() and the
package's marshalling make -- TEST INFRASTRUCTURE ONLY.

Installed as ``torch`` in a child process (see dryrun.py) together with the emulated library,
it lets the benchmark's and the smoke check's own code run end to end on the CPU: "device"
tensors are numpy arrays whose data pointers the emulated library reads and writes.
"""
from __future__ import annotations

import time
import types

import numpy as np

int32 = np.dtype(np.int32)
int64 = np.dtype(np.int64)
uint8 = np.dtype(np.uint8)


class device:
    def __init__(self, spec="cuda:0"):
        self.spec = str(spec)
        self.type = self.spec.split(":")[0]

    def __repr__(self):
        return "device(%r)" % self.spec


def _np_dtype(d):
    return np.dtype(d) if d is not None else np.dtype(np.float32)


class Tensor:
    is_cuda = True

    def __init__(self, a, dev=None):
        self.a = a
        self.device = dev or device("cuda:0")

    @property
    def dtype(self):
        return self.a.dtype

    @property
    def shape(self):
        return self.a.shape

    def numel(self):
        return int(self.a.size)

    def is_contiguous(self):
        return bool(self.a.flags.c_contiguous)

    def data_ptr(self):
        return int(self.a.ctypes.data)

    def __getitem__(self, k):
        return Tensor(self.a[k], self.device)

    def __len__(self):
        return len(self.a)

    def clone(self):
        return Tensor(self.a.copy(), self.device)

    def contiguous(self):
        return self if self.is_contiguous() else self.clone()

    def cpu(self):
        return self

    def numpy(self):
        return self.a

    def to(self, dev):
        return Tensor(np.ascontiguousarray(self.a).copy(), dev if isinstance(dev, device) else device(dev))

    def copy_(self, other):
        self.a[...] = other.a
        return self

    def fill_(self, v):
        self.a.fill(v)
        return self

    def view(self, dt):
        return Tensor(self.a.view(dt), self.device)

    def max(self):
        return Tensor(np.asarray(self.a.max()))

    def item(self):
        return self.a.item()


def _aligned_empty(n, dt):
    dt = _np_dtype(dt)
    nbytes = int(n) * dt.itemsize
    raw = np.empty(nbytes + 256, np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw[off:off + nbytes].view(dt)


def empty(n, dtype=None, device=None):
    a = _aligned_empty(n, dtype)
    a.view(np.uint8).fill(0xA5)   # device memory holds anything
    return Tensor(a, device)


def zeros(n, dtype=None, device=None):
    a = _aligned_empty(n, dtype)
    a.fill(0)
    return Tensor(a, device)


def empty_like(t):
    return empty(t.numel(), t.dtype, t.device)


def from_numpy(a):
    return Tensor(a)


def tensor(values, dtype=None, device=None):
    a = _aligned_empty(len(values), dtype)
    a[...] = np.asarray(values, dtype=a.dtype)
    return Tensor(a, device)


def arange(a, b=None, device=None, dtype=None):
    lo, hi = (0, a) if b is None else (a, b)
    return Tensor(np.arange(lo, hi, dtype=_np_dtype(dtype) if dtype is not None else np.int64), device)


def equal(x, y):
    return bool(x.a.shape == y.a.shape and np.array_equal(x.a, y.a))


class _Stream:
    cuda_stream = 0

    def synchronize(self):
        pass


class _Event:
    def __init__(self, enable_timing=False):
        self.t = None

    def record(self, stream=None):
        self.t = time.perf_counter()

    def elapsed_time(self, end):
        return (end.t - self.t) * 1e3


class _Props:
    gcnArchName = "emulated"
    multi_processor_count = 4


cuda = types.SimpleNamespace(
    is_available=lambda: True,
    synchronize=lambda *a, **k: None,
    empty_cache=lambda: None,
    current_stream=lambda *a, **k: _Stream(),
    Event=_Event,
    get_device_properties=lambda i: _Props(),
    device_count=lambda: 1,
)
