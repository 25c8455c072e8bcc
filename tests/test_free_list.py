"""The request server's arena bookkeeping (free_list.hpp), built for the
host with g++ and driven by random allocation sequences against a plain
model: blocks never overlap and stay inside the arena, the lowest fitting
address is chosen, used bytes add up, and freed neighbours merge so that an
empty arena is one block again."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GRAIN = 256
NONE = ctypes.c_size_t(-1).value


@pytest.fixture(scope="module")
def fl(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fl") / "libfl.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", os.path.join(HERE, "free_list_host.cpp"),
                    "-o", out], check=True)
    lib = ctypes.CDLL(out)
    sz = ctypes.c_size_t
    for name, res, args in (("fl_reset", None, [sz]), ("fl_alloc", sz, [sz]), ("fl_release", None, [sz, sz]),
                            ("fl_used", sz, []), ("fl_size", sz, []), ("fl_free_blocks", sz, []),
                            ("fl_largest_free", sz, [])):
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    return lib


def _round(b):
    return max(GRAIN, -(-b // GRAIN) * GRAIN)


def _first_fit(live, size, need):
    """Lowest offset where `need` bytes fit between live blocks."""
    pos = 0
    for off, length in sorted(live.values()):
        if off - pos >= need:
            return pos
        pos = max(pos, off + length)
    return pos if size - pos >= need else None


@pytest.mark.parametrize("seed", range(6))
def test_random_sequences_match_the_model(fl, seed):
    rng = np.random.default_rng(seed)
    size = int(rng.integers(1, 64)) * 4096 + int(rng.integers(0, 300))
    fl.fl_reset(size)
    size_r = -(-size // GRAIN) * GRAIN
    assert fl.fl_size() == size_r
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            key = list(live)[int(rng.integers(0, len(live)))]
            off, length = live.pop(key)
            fl.fl_release(off, length)
        else:
            req = int(rng.integers(1, size_r // 4 + 2))
            off = fl.fl_alloc(req)
            want = _first_fit(live, size_r, _round(req))
            if want is None:
                assert off == NONE
                continue
            assert off == want, (step, off, want)
            live[step] = (off, _round(req))
        assert fl.fl_used() == sum(l for _, l in live.values())
        spans = sorted(live.values())
        for (a, la), (b, _) in zip(spans, spans[1:]):
            assert a + la <= b
        assert all(o + l <= size_r for o, l in spans)
    for off, length in live.values():
        fl.fl_release(off, length)
    assert fl.fl_used() == 0 and fl.fl_free_blocks() == 1 and fl.fl_largest_free() == size_r
    assert fl.fl_alloc(size_r) == 0


def test_rounding_and_exhaustion(fl):
    fl.fl_reset(1000)                      # rounds up to 1024
    assert fl.fl_size() == 1024
    assert fl.fl_alloc(1) == 0             # one granule
    assert fl.fl_alloc(257) == 256         # two granules
    assert fl.fl_alloc(256) == 768
    assert fl.fl_alloc(1) == NONE          # full
    fl.fl_release(256, 257)
    assert fl.fl_alloc(512) == 256         # the freed hole
    assert fl.fl_used() == 1024
