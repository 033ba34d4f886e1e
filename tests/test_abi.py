"""The C-ABI library loads and exports every function include/vcipher.h
declares; host-only logic (key bytes, validation before any device call)
behaves as documented.  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vcipher.h")
LIB = os.path.join(ROOT, "paper_2505_07158_amd", "libvcipher.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"\b([A-Za-z_]\w*)\s*\([^;{}()]*(?:\([^)]*\)[^;{}()]*)*\)\s*;", text)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2505_07158_amd.build as b
        b.build()
    return C.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("cipher_init", "encrypt_frames", "decrypt_frames", "cipher_destroy"):
        assert required in names
    assert len(names) >= 15


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_functions(lib):
    lib.vc_protocol_version.restype = C.c_uint32
    assert lib.vc_protocol_version() == 1
    lib.vc_strerror.restype = C.c_char_p
    for code in range(-7, 1):
        assert lib.vc_strerror(code)
    lib.vc_kernel_name.restype = C.c_char_p
    assert [lib.vc_kernel_name(k).decode() for k in range(5)] == [
        "sha256_subframes", "lhcs_chain", "lhcs_keygen", "confuse_xor_enc", "confuse_xor_dec"]


def test_key_from_bytes_agrees_with_oracle():
    from paper_2505_07158_amd import vcipher as V
    rng = np.random.default_rng(3)
    for _ in range(50):
        kb = rng.bytes(32)
        k = V.vc_key_from_bytes(kb, -1.0, 32)
        np.testing.assert_array_equal([k.x0, k.y0, k.z0, k.w0], oracle.key_from_bytes(kb))
        assert k.gamma == -1.0 and k.n == 32


@pytest.mark.parametrize("gamma,n", [(-1.6, 32), (-0.05, 32), (-1.0, 0), (-1.0, 1025), (float("nan"), 4)])
def test_invalid_keys_rejected_before_device_use(gamma, n):
    from paper_2505_07158_amd import vcipher as V
    with pytest.raises(V.VcError) as e:
        V.vc_key_from_bytes(bytes(32), gamma, n)
    assert e.value.status == V.VC_EINVAL
    key = V.VcKey(1.0, 2.0, 3.0, 4.0, gamma, n)
    with pytest.raises(V.VcError) as e:
        V.cipher_init(key, 1, 0)
    assert e.value.status == V.VC_EINVAL


def test_nonfinite_key_and_zero_streams_rejected():
    from paper_2505_07158_amd import vcipher as V
    for key, streams in ((V.VcKey(float("inf"), 0, 0, 0, -1.0, 4), 1), (V.VcKey(1, 2, 3, 4, -1.0, 4), 0)):
        with pytest.raises(V.VcError) as e:
            V.cipher_init(key, streams, 0)
        assert e.value.status == V.VC_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the Python binding mirrors has the header's size and
    field offsets (a host program built with gcc prints them)."""
    import shutil
    import subprocess
    from paper_2505_07158_amd import vcipher as V
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    mirrored = {"vc_key": V.VcKey, "vc_shape": V.VcShape, "vc_request": V.VcRequest,
                "vc_completion": V.VcCompletion, "vc_sched_config": V.VcSchedConfig,
                "vc_sched_stats": V.VcSchedStats, "vc_server_config": V.VcServerConfig}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vcipher.h"', "int main(void) {"]
    for cname, py in mirrored.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, value = ln.split()
        got[(cname, field)] = int(value)
    for cname, py in mirrored.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_constants_match_the_header(tmp_path):
    """The binding's status codes, prepared-batch modes and serving kinds
    have the header's values (a host program built with gcc prints them)."""
    import shutil
    import subprocess
    from paper_2505_07158_amd import serving
    from paper_2505_07158_amd import vcipher as V
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    names = ["VC_OK", "VC_EINVAL", "VC_ENOMEM", "VC_EDEVICE", "VC_EORDER", "VC_ENONFINITE", "VC_EBUSY",
             "VC_PREP_ENCRYPT", "VC_PREP_DECRYPT", "VC_PREP_HASH", "VC_PREP_ENCRYPT_HASHED"]
    kinds = ["VC_REQ_ENCRYPT", "VC_REQ_DECRYPT", "VC_BATCH_HASH"]
    lines = ["#include <stdio.h>", '#include "vcipher.h"', "int main(void) {"]
    lines += [f'printf("{nm} %d\\n", (int){nm});' for nm in names + kinds]
    lines += ["return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict((a, int(b)) for a, b in (ln.split() for ln in subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()))
    for nm in names:
        assert got[nm] == getattr(V, nm), nm
    # the serving binding's kind strings are indexed by the header's kinds
    assert [serving.KINDS[got[k]] for k in kinds] == ["enc", "dec", "hash"]
    assert V.PREP_MODES == {"encrypt": got["VC_PREP_ENCRYPT"], "decrypt": got["VC_PREP_DECRYPT"],
                            "hash": got["VC_PREP_HASH"], "encrypt_hashed": got["VC_PREP_ENCRYPT_HASHED"]}


def test_pointer_reachable_refuses_host_memory(lib):
    """vc_pointer_reachable: pageable host memory, NULL and empty ranges are
    not device-addressable (with or without a GPU)."""
    lib.vc_pointer_reachable.argtypes = [C.c_void_p, C.c_size_t]
    lib.vc_pointer_reachable.restype = C.c_int
    buf = (C.c_uint8 * 64)()
    assert lib.vc_pointer_reachable(C.cast(buf, C.c_void_p), 64) == 0
    assert lib.vc_pointer_reachable(None, 16) == 0
    assert lib.vc_pointer_reachable(C.cast(buf, C.c_void_p), 0) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus above 1 exits with a message (no GPU
    is touched)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
