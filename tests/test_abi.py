"""C-ABI surface, host only: the library loads, exports every symbol that
include/*.h declares, and rejects bad arguments before any GPU call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbessel.h", "lbessel_serve.h")]


def declared_symbols():
    found = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        found.update(re.findall(r"\b(lbessel_\w+)\s*\(", text))
    return sorted(found)


def test_headers_are_the_whole_include_dir():
    names = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert names == sorted(os.path.basename(h) for h in HEADERS)


@pytest.fixture(scope="module")
def lib():
    import paper_2409_08729_amd as lb
    return lb.lib()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(lib, s), s


def test_version_and_status(lib):
    assert lib.lbessel_abi_version() == 1
    assert lib.lbessel_status_string(0) == b"ok"
    assert lib.lbessel_status_string(-1) == b"invalid argument"
    assert lib.lbessel_status_string(-2) == b"HIP launch failure"
    assert lib.lbessel_status_string(-4) == b"request larger than the server arena"
    assert lib.lbessel_status_string(-5) == b"timed out"
    assert lib.lbessel_status_string(12345) == b"unknown status"


@pytest.mark.parametrize("name", ["lbessel_log_iv_f64", "lbessel_log_iv_f32",
                                  "lbessel_log_kv_f64", "lbessel_log_kv_f32",
                                  "lbessel_log_kv_integral_f64"])
def test_forward_argument_checks(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, 0, None) == 0          # n = 0: nothing to do
    assert fn(None, None, None, -1, None) == -1        # n < 0
    assert fn(None, None, None, 16, None) == -1        # NULL with n > 0


@pytest.mark.parametrize("name", ["lbessel_log_iv_grad_x_f64", "lbessel_log_kv_grad_x_f64",
                                  "lbessel_log_iv_grad_x_f32", "lbessel_log_kv_grad_x_f32"])
def test_grad_argument_checks(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, None, 0, None) == 0
    assert fn(None, None, None, None, 8, None) == -1


def test_vmf_argument_checks(lib):
    assert lib.lbessel_vmf_log_norm_f64(None, 1.5, None, 0, None) == -1   # p < 2
    assert lib.lbessel_vmf_log_norm_f64(None, float("nan"), None, 0, None) == -1
    assert lib.lbessel_vmf_log_norm_f64(None, 3.0, None, 0, None) == 0
    assert lib.lbessel_vmf_log_norm_f64(None, 3.0, None, 5, None) == -1
    assert lib.lbessel_vmf_log_norm_grad_f64(None, 1.0, None, 0, None) == -1


def test_diagnostic_argument_checks(lib):
    assert lib.lbessel_classify(2, 64, None, None, None, 0, None) == -1     # bad kind
    assert lib.lbessel_classify(0, 16, None, None, None, 0, None) == -1     # bad precision
    assert lib.lbessel_eval_branch_f64(0, 3, None, None, None, 0, None) == -1
    assert lib.lbessel_eval_branch_f32(2, 0, None, None, None, 0, None) == -1
    assert lib.lbessel_eval_branch_f32(0, 0, None, None, None, 0, None) == 0
    assert lib.lbessel_eval_ungrouped(1, 64, None, None, None, 0, None) == 0
    assert lib.lbessel_k_terms(64, None, None, None, 0, None) == 0
    assert lib.lbessel_k_terms(32, None, None, None, -1, None) == -1
    assert lib.lbessel_k_terms(64, None, None, None, 5, None) == -1
    assert lib.lbessel_k_terms(16, None, None, None, 0, None) == -1
    assert lib.lbessel_elementary_f64(6, None, None, 0, None) == -1
    assert lib.lbessel_elementary_f64(5, None, None, 0, None) == 0
    assert lib.lbessel_elementary_f64(0, None, None, 0, None) == 0
    assert lib.lbessel_elementary_f64(3, None, None, 4, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2409_08729_amd as lb
    with pytest.raises(lb.LbesselError):
        lb.log_iv(torch.ones(4, dtype=torch.float64), torch.ones(4, dtype=torch.float64))


def test_segment_and_fit_argument_checks(lib):
    lib.lbessel_segment_tiles.restype = ctypes.c_int64
    lib.lbessel_segment_tiles.argtypes = [ctypes.c_int64]
    assert [lib.lbessel_segment_tiles(n) for n in (0, 1, 1024, 1025)] == [0, 1, 1, 2]
    assert lib.lbessel_segment_tiles(-1) == -1
    assert lib.lbessel_eval_segments(0, 64, None, 0, 0, None) == 0         # empty batch
    assert lib.lbessel_eval_segments(2, 64, None, 0, 0, None) == -1        # bad kind
    assert lib.lbessel_eval_segments(0, 64, None, 3, 5, None) == -1        # NULL table
    fake = ctypes.c_void_p(1 << 20)     # never read: every call below fails first
    assert lib.lbessel_eval_segments_inline(0, 64, fake, 33, 5, None) == -1  # > 32 entries
    assert lib.lbessel_eval_segments_inline(0, 16, fake, 3, 5, None) == -1
    assert lib.lbessel_eval_segments_inline(0, 64, None, 3, 5, None) == -1
    assert lib.lbessel_eval_segments_inline(0, 64, None, 0, 0, None) == 0
    lib.lbessel_vmf_fit_f32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p]
    assert lib.lbessel_vmf_fit_f32(None, 0, 8, None, None, 0, None) == -1  # n < 1
    assert lib.lbessel_vmf_fit_f32(None, 10, 8, None, None, 0, None) == -1


def test_noalloc_fit_size_checks(lib):
    """The no-allocation fit rejects NULL pointers and sizes beyond its static
    buffer on the host, before touching a device."""
    fn = lib.lbessel_vmf_fit_f32_noalloc
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                   ctypes.c_void_p]
    fn.restype = ctypes.c_int
    fake = ctypes.c_void_p(1 << 20)    # never dereferenced: every call below fails first
    assert fn(None, 10, 8, fake, None) == -1
    assert fn(fake, 10, 8, None, None) == -1
    assert fn(fake, 0, 8, fake, None) == -1                 # n < 1
    assert fn(fake, 10, 1, fake, None) == -1                # p < 2
    assert fn(fake, 2_000_000, 32768, fake, None) == -7     # 26.2 MB > 24 MiB
    assert fn(fake, 3_000_000, 2048, fake, None) == -7
    assert fn(fake, 10, 1 << 40, fake, None) == -7          # p alone exceeds the buffer
    assert fn(fake, 1 << 40, 8, fake, None) == -7
    assert lib.lbessel_status_string(-7) == b"request larger than the static buffer"
    lib.lbessel_vmf_fit_workspace.restype = ctypes.c_int64
    lib.lbessel_vmf_fit_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64]
    # the documented limits: p = 32768 to about 1.0e6 rows, p = 2048 to 2.6e6
    cap = 24 << 20
    assert lib.lbessel_vmf_fit_workspace(1_015_807, 32768) <= cap
    assert lib.lbessel_vmf_fit_workspace(1_015_808, 32768) > cap
    assert lib.lbessel_vmf_fit_workspace(2_619_391, 2048) <= cap
    assert lib.lbessel_vmf_fit_workspace(2_619_392, 2048) > cap


def test_server_needs_a_device():
    import torch
    from paper_2409_08729_amd import serve
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible: covered by the GPU serving tests")
    with pytest.raises(Exception, match="no usable device"):
        serve.Server()


def test_server_config_layout_and_defaults(lib, tmp_path):
    """The binding's Config mirrors lbessel_server_config_t (field offsets and
    size from the C compiler), and the library's defaults are the documented
    ones."""
    import shutil
    import subprocess
    from paper_2409_08729_amd import serve
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [name for name, _ in serve.Config._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbessel_serve.h"\n'
                   "int main(void) {\n"
                   '  printf("%zu", sizeof(lbessel_server_config_t));\n'
                   + "".join(f'  printf(" %zu", offsetof(lbessel_server_config_t, {f}));\n'
                             for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(t) for t in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(serve.Config)
    assert got[1:] == [getattr(serve.Config, f).offset for f in fields]
    cfg = serve.Config()
    serve._lib().lbessel_server_default_config(ctypes.byref(cfg))
    assert (cfg.arena_bytes, cfg.streams, cfg.mode, cfg.max_batch_requests, cfg.max_batch_elems,
            cfg.poll_us, cfg.solo_elems) == (2 << 30, 8, 0, 64, 1 << 18, 0, 1 << 16)
