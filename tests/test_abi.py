"""Host-side checks of the C-ABI library (no GPU needed).

* libppc.so loads and exports every function declared in include/*.h.
* Argument validation that happens before any HIP call returns the
  documented status codes.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ppc_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2412_16370_amd as ppc

    return ppc.lib()


def test_header_declares_the_plain_calls():
    names = declared_functions()
    for w in (8, 16, 32, 64):
        assert "ppc_pospopcnt%d" % w in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(lib, name):
    assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(6):
        assert lib.ppc_status_string(code) != b"PPC_UNKNOWN"
    assert lib.ppc_status_string(5).startswith(b"PPC_ETIMEDOUT")
    assert lib.ppc_status_string(99) == b"PPC_UNKNOWN"


def test_struct_layouts_match_the_header():
    """The binding's ctypes structs have the sizes and field offsets of the
    C structs in include/ppc.h (natural alignment, no packing)."""
    import paper_2412_16370_amd as ppc

    assert ctypes.sizeof(ppc.ppc_desc) == 32
    assert ctypes.sizeof(ppc.ppc_server_cfg) == 32
    assert ppc.ppc_server_cfg.inflight_bytes.offset == 16
    assert ppc.ppc_server_cfg.batch_timeout_us.offset == 28
    assert ctypes.sizeof(ppc.ppc_request) == 32
    assert ctypes.sizeof(ppc.ppc_result) == 32 + 64 * 8
    assert ppc.PPC_ETIMEDOUT == 5


def test_invalid_arguments_rejected_before_any_device_work(lib):
    fake = 0x1000  # never dereferenced: validation fails first
    assert lib.ppc_pospopcnt(12, fake, fake, 10, None) == 1
    assert lib.ppc_pospopcnt(0, fake, fake, 10, None) == 1
    assert lib.ppc_pospopcnt(16, None, fake, 10, None) == 1
    assert lib.ppc_pospopcnt(16, fake + 4, fake, 10, None) == 1   # counts not 8-aligned
    assert lib.ppc_pospopcnt16(None, fake, 10, None) == 1
    assert lib.ppc_pospopcnt64(fake, None, 10, None) == 1         # NULL buf, nbytes > 0


def test_empty_input_is_a_no_op(lib):
    for w in (8, 16, 32, 64):
        assert lib.ppc_pospopcnt(w, 0x1000, None, 0, None) == 0


def test_plain_geometry_validation(lib):
    assert lib.ppc_set_plain_geometry(0, 3) == 1
    assert lib.ppc_set_plain_geometry(0, 1) == 1
    assert lib.ppc_set_plain_geometry(0, 2) == 0
    assert lib.ppc_set_plain_geometry(0, 16) == 1
    assert lib.ppc_set_plain_geometry(1 << 25, 4) == 1
    assert lib.ppc_set_plain_geometry(0, 4) == 0
    assert lib.ppc_set_plain_geometry(0, 8) == 0


def test_roofline_validation(lib):
    assert lib.ppc_read_roofline(None, 0x1000, 16384, None) == 1
    assert lib.ppc_read_roofline(0x1000, 0x1001, 16384, None) == 1
    assert lib.ppc_read_roofline(0x1000, 0x1000, 100, None) == 1


def test_stream_and_popcount_validation(lib):
    fake = 0x1000
    assert lib.ppc_pospopcnt_at(0, fake, fake, 10, 3, None) == 1   # width 0 is not a width
    assert lib.ppc_pospopcnt_at(24, fake, fake, 10, 3, None) == 1
    assert lib.ppc_pospopcnt_at(16, fake + 2, fake, 10, 3, None) == 1
    assert lib.ppc_pospopcnt_at(16, fake, None, 0, 3, None) == 0
    assert lib.ppc_popcount(None, fake, 10, None) == 1
    assert lib.ppc_popcount(fake + 4, fake, 10, None) == 1
    assert lib.ppc_popcount(fake, None, 10, None) == 1
    assert lib.ppc_popcount(fake, None, 0, None) == 0


def test_noalloc_batch_validation(lib):
    # checked before any HIP call: too many arrays, NULL or misaligned tables
    assert lib.ppc_batch_noalloc(None, 65537, None, None) == 1
    assert lib.ppc_batch_noalloc(0x1000, 65537, None, None) == 1
    assert lib.ppc_batch_noalloc(None, 3, None, None) == 1
    assert lib.ppc_batch_noalloc(0x1004, 3, None, None) == 1
    assert lib.ppc_batch_noalloc(0x1000, 3, 0x1002, None) == 1


def test_binding_bounds_nbytes_by_the_tensor():
    """The binding refuses a byte count larger than the tensor it is given,
    so a length mistake cannot turn into a read past the buffer."""
    torch = pytest.importorskip("torch")
    import paper_2412_16370_amd as ppc

    t = torch.zeros(10, dtype=torch.uint8)
    assert ppc._nbytes(t, None) == 10
    assert ppc._nbytes(t, 7) == 7
    assert ppc._nbytes(torch.zeros(3, dtype=torch.int64), None) == 24
    with pytest.raises(ValueError):
        ppc._nbytes(t, 11)
    with pytest.raises(ValueError):
        ppc._nbytes(t, -1)
    with pytest.raises(ValueError):
        ppc._nbytes(0x1000, None)   # a raw address needs its length
    assert ppc._nbytes(0x1000, 5) == 5


def test_library_and_torch_share_one_hip_runtime():
    """torch bundles its own HIP runtime under the soname libppc.so links
    against.  Loading the library before torch (here: a call that needs no
    tensor) must still leave one runtime in the process, or torch's streams
    are unknown to the library's launches."""
    import ast
    import subprocess
    import sys

    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2412_16370_amd as ppc\n"
        "ppc.lib().ppc_version()\n"
        "import torch\n"
        "print(sorted({ln.split()[-1] for ln in open('/proc/self/maps') if 'libamdhip64' in ln}))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    runtimes = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(runtimes) == 1, runtimes
