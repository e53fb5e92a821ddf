"""Helpers for GPU tests: place host arrays at chosen byte offsets in device
memory, call the C ABI with raw pointers, check guard bytes around outputs."""
from __future__ import annotations

import sys

import numpy as np
import torch

GUARD = 64          # guard bytes on each side of an output region
CANARY = 0xA5


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


class DeviceBytes:
    """A host byte array copied to device memory at `offset` bytes past a
    256-byte aligned address."""

    def __init__(self, data: np.ndarray, offset: int = 0):
        raw = np.ascontiguousarray(data).view(np.uint8).reshape(-1)
        self.nbytes = raw.size
        self.buf = torch.zeros(raw.size + offset + 512, dtype=torch.uint8, device="cuda")
        base = (self.buf.data_ptr() + 255) & ~255
        self.start = base - self.buf.data_ptr() + offset
        if raw.size:
            self.buf[self.start:self.start + raw.size] = torch.from_numpy(raw.copy()).cuda()
        self.ptr = self.buf.data_ptr() + self.start


class DeviceOut:
    """An output region of `cap_bytes` bytes at `offset` past a 256-byte
    aligned address, surrounded by canary bytes (also filling the region)."""

    def __init__(self, cap_bytes: int, offset: int = 0):
        self.cap_bytes = cap_bytes
        self.buf = torch.full((cap_bytes + offset + 2 * GUARD + 512,), CANARY, dtype=torch.uint8, device="cuda")
        base = (self.buf.data_ptr() + 255) & ~255
        self.start = base - self.buf.data_ptr() + GUARD + offset
        self.ptr = self.buf.data_ptr() + self.start

    def host(self) -> np.ndarray:
        return self.buf.cpu().numpy()

    def region(self, h: np.ndarray) -> np.ndarray:
        return h[self.start:self.start + self.cap_bytes]

    def check_guards(self, h: np.ndarray, written_bytes: int | None = None):
        """Nothing outside [ptr, ptr+cap) changed; with written_bytes, nothing
        in [ptr+written, ptr+cap) either."""
        assert np.all(h[:self.start] == CANARY), "write before the output region"
        assert np.all(h[self.start + self.cap_bytes:] == CANARY), "write past the output capacity"
        if written_bytes is not None:
            assert np.all(h[self.start + written_bytes:self.start + self.cap_bytes] == CANARY), \
                "write past the reported count"
