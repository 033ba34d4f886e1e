"""The C ABI used from plain C.  tests/c_abi/roundtrip.c: hipMalloc'ed
buffers, encrypt_frames / decrypt_frames of two streams of different shapes
in one call, every byte, hash and chain state equal to the oracle's, and a
pageable hash buffer refused before anything is enqueued.
tests/c_abi/serve.c: the serving loop (vc_server_*) over four streams of two
resolutions, out-of-order submission with hash-first batches, then a reset
and a trace replay; every served frame equal to the oracle's or to the
plaintext."""
import importlib.util
import os
import subprocess

import pytest

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def driver(name: str = "roundtrip") -> str:
    path = os.path.join(HERE, "c_abi", name)
    if not os.path.exists(path):
        spec = importlib.util.spec_from_file_location("build_driver", os.path.join(HERE, "c_abi", "build_driver.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        path = mod.build_one(name)
    return path


def test_c_program_round_trip_matches_oracle():
    require_gpu()
    r = subprocess.run([driver()], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "roundtrip ok" in r.stdout


def test_c_program_serving_loop_matches_oracle():
    require_gpu()
    r = subprocess.run([driver("serve")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "serve ok" in r.stdout
