"""The C-ABI library loads and exports every symbol its header declares, and
its host-side argument checks behave as documented (no GPU needed: invalid
calls are rejected before anything touches the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastvol.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_27210_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        from paper_2604_27210_amd import build
        build.build()
    return N.load()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("fv_price", "fv_implied_vol", "fv_greeks", "fv_implied_vol_backward",
                 "fv_implied_vol_chains", "fv_normalised_black", "fv_autotune",
                 "fv_set_launch", "fv_get_launch", "fv_last_error", "fv_version"):
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    from paper_2604_27210_amd import _native as N
    fns = declared_functions()
    missing = [f for f in fns if not hasattr(lib, f)]
    assert not missing, missing
    assert set(fns) == set(N.EXPORTS)


def test_version_and_error_paths(lib):
    from paper_2604_27210_amd import _native as N
    assert lib.fv_version() == 1
    # invalid launch shapes and kernel ids
    assert lib.fv_set_launch(1, 96, 1) == N.FV_E_INVALID_ARG
    assert b"shape" in lib.fv_last_error()
    assert lib.fv_set_launch(99, 256, 1) == N.FV_E_INVALID_ARG
    b, q = ctypes.c_int(), ctypes.c_int()
    assert lib.fv_get_launch(1, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
    assert b.value % 64 == 0 and q.value >= 1
    # Halley shapes whose LDS queue would exceed 64 KiB are refused; the
    # shape in force is left as it was
    for kern in (2, 6):
        assert lib.fv_get_launch(kern, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
        saved = (b.value, q.value)
        assert lib.fv_set_launch(kern, 512, 16) == N.FV_E_INVALID_ARG
        assert b"LDS" in lib.fv_last_error()
        assert lib.fv_get_launch(kern, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
        assert (b.value, q.value) == saved
    assert lib.fv_get_launch(0, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
    saved = (b.value, q.value)
    assert lib.fv_set_launch(0, 512, 16) == N.FV_OK  # no queue: any valid shape
    assert lib.fv_set_launch(0, *saved) == N.FV_OK
    # invalid model / solver / NULL outputs are refused before any launch
    qs = N.FvQuotes(4, N.FvArg(None, 1.0), N.FvArg(None, 100.0), N.FvArg(None, 100.0),
                    N.FvArg(None, 1.0), N.FvArg(None, 0.0), N.FvArg(None, 0.0), None, 1)
    dummy = ctypes.c_void_p(16)
    assert lib.fv_implied_vol(7, 0, ctypes.byref(qs), dummy, None, None, None) == N.FV_E_INVALID_ARG
    assert b"model" in lib.fv_last_error()
    assert lib.fv_implied_vol(2, 9, ctypes.byref(qs), dummy, None, None, None) == N.FV_E_INVALID_ARG
    assert lib.fv_implied_vol(2, 0, ctypes.byref(qs), None, None, None, None) == N.FV_E_INVALID_ARG
    assert b"sigma_out" in lib.fv_last_error()
    assert lib.fv_implied_vol(2, 0, None, dummy, None, None, None) == N.FV_E_INVALID_ARG
    bad_n = N.FvQuotes(-1, N.FvArg(None, 1.0), N.FvArg(None, 100.0), N.FvArg(None, 100.0),
                       N.FvArg(None, 1.0), N.FvArg(None, 0.0), N.FvArg(None, 0.0), None, 1)
    assert lib.fv_price(2, ctypes.byref(bad_n), N.FvArg(None, 0.2), dummy, None) == N.FV_E_INVALID_ARG
    bad_flag = N.FvQuotes(4, N.FvArg(None, 1.0), N.FvArg(None, 100.0), N.FvArg(None, 100.0),
                          N.FvArg(None, 1.0), N.FvArg(None, 0.0), N.FvArg(None, 0.0), None, 0)
    assert lib.fv_price(2, ctypes.byref(bad_flag), N.FvArg(None, 0.2), dummy, None) == N.FV_E_INVALID_ARG
    huge = N.FvQuotes((1 << 31) * 64, N.FvArg(None, 1.0), N.FvArg(None, 100.0),
                      N.FvArg(None, 100.0), N.FvArg(None, 1.0), N.FvArg(None, 0.0),
                      N.FvArg(None, 0.0), None, 1)
    assert lib.fv_implied_vol(2, 0, ctypes.byref(huge), dummy, None, None, None) == N.FV_E_INVALID_ARG
    assert b"2^31" in lib.fv_last_error()
    assert lib.fv_implied_vol_chains(0, None, dummy, None, None) == N.FV_E_INVALID_ARG
    assert lib.fv_normalised_black(-1, None, None, None, None, None) == N.FV_E_INVALID_ARG
    # n == 0 is a no-op
    zero = N.FvQuotes(0, N.FvArg(None, 1.0), N.FvArg(None, 100.0), N.FvArg(None, 100.0),
                      N.FvArg(None, 1.0), N.FvArg(None, 0.0), N.FvArg(None, 0.0), None, 1)
    assert lib.fv_implied_vol(2, 0, ctypes.byref(zero), dummy, None, None, None) == N.FV_OK
    assert lib.fv_implied_vol(2, 0, ctypes.byref(zero), None, None, None, None) == N.FV_OK
    assert lib.fv_price(2, ctypes.byref(zero), N.FvArg(None, 0.2), None, None) == N.FV_OK


def test_library_is_gfx950_code():
    from paper_2604_27210_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("not built")
    blob = open(N.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_tuning_file_validation_and_shape_query(lib, tmp_path):
    """Malformed tuning files are refused before any device is touched, and
    the shape query reports the configured shape narrowed for small batches."""
    from paper_2604_27210_amd import _native as N
    bad = {
        "empty": "",
        "not ours": "{}",
        "version": '{"format": "fastvol-tuning", "version": 2, "arch": "x", "entries": []}',
        "bucket": '{"format": "fastvol-tuning", "version": 1, "arch": "x", "entries": '
                  '[{"kernel": 1, "model": 2, "bucket": 9, "block": 128, "qpt": 1}]}',
        "lds": '{"format": "fastvol-tuning", "version": 1, "arch": "x", "entries": '
               '[{"kernel": 2, "model": 2, "bucket": 3, "block": 512, "qpt": 16}]}',
        "block": '{"format": "fastvol-tuning", "version": 1, "arch": "x", "entries": '
                 '[{"kernel": 1, "model": 2, "bucket": 3, "block": 96, "qpt": 1}]}',
        "field": '{"format": "fastvol-tuning", "version": 1, "arch": "x", "entries": '
                 '[{"kernel": 1, "model": 2, "block": 128, "qpt": 1}]}',
        "wide": '{"format": "fastvol-tuning", "version": 1, "arch": "x", "entries": '
                '[{"kernel": 1, "model": 2, "bucket": 3, "block": 4294967552, "qpt": 1}]}',
    }
    for name, text in bad.items():
        p = tmp_path / (name + ".json")
        p.write_text(text)
        assert lib.fv_tuning_load(str(p).encode()) == N.FV_E_INVALID_ARG, name
    assert lib.fv_tuning_load(str(tmp_path / "missing.json").encode()) == N.FV_E_INVALID_ARG
    assert lib.fv_tuning_load(None) == N.FV_E_INVALID_ARG
    assert lib.fv_tuning_save(None) == N.FV_E_INVALID_ARG
    assert lib.fv_tuning_reset() == N.FV_OK
    b, q = ctypes.c_int(), ctypes.c_int()
    assert lib.fv_launch_shape(1, 2, 0, ctypes.byref(b), ctypes.byref(q)) == N.FV_E_INVALID_ARG
    assert lib.fv_launch_shape(9, 2, 10, ctypes.byref(b), ctypes.byref(q)) == N.FV_E_INVALID_ARG
    gb, gq = ctypes.c_int(), ctypes.c_int()
    assert lib.fv_get_launch(1, ctypes.byref(gb), ctypes.byref(gq)) == N.FV_OK
    # a batch far larger than the device: the configured shape as is
    assert lib.fv_launch_shape(1, 2, 1 << 30, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
    assert (b.value, q.value) == (gb.value, gq.value)
    # one quote: one-wave workgroups, one quote per thread
    assert lib.fv_launch_shape(1, 2, 1, ctypes.byref(b), ctypes.byref(q)) == N.FV_OK
    assert (b.value, q.value) == (64, 1)


def test_missing_library_raises_instead_of_falling_back(tmp_path):
    """With no built library the binding raises: there is no CPU path to
    fall back to.  Run in a child process so this process keeps its loaded
    library."""
    import subprocess
    import sys
    code = ("import paper_2604_27210_amd as fv\n"
            "from paper_2604_27210_amd import _native as N\n"
            "try:\n"
            "    N.load()\n"
            "except N.FastvolError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('loaded a library that does not exist')\n")
    env = dict(os.environ, FASTVOL_LIBRARY=str(tmp_path / "absent" / "libfastvol.so"))
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "raised: libfastvol.so is not built" in res.stdout


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU and says so for --gpus N > 1 (it exits
    before touching any device)."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "measures one GPU" in res.stdout + res.stderr


def test_svi_workspace_size_and_small_workspace(lib):
    """fv_svi_workspace_size follows the documented layout, and a step with
    a smaller workspace is refused before anything is launched (the arrays
    below are never dereferenced)."""
    from paper_2604_27210_amd import _native as N
    assert lib.fv_svi_workspace_size(None) == N.FV_E_INVALID_ARG
    fake = 0x1000
    for n_mat, n in ((1, 1), (7, 64), (7, 65), (7529, 2080919)):
        ch = N.FvChains(1, n_mat, n, fake, fake, fake, fake, fake, None, fake, fake)
        prob = N.FvSviProblem(ch, fake, 1e-2, 0.9, 0.999, 1e-8)
        need = lib.fv_svi_workspace_size(ctypes.byref(prob))
        assert need == 2 + 8 * n_mat + (n_mat + 3) // 4 + 6 * ((n + 63) // 64 + n_mat)
        v = ctypes.c_void_p(fake)
        rc = lib.fv_svi_adam_step(ctypes.byref(prob), v, v, v, v, v, v, need - 1, None, 0, None)
        assert rc == N.FV_E_INVALID_ARG
        assert b"workspace" in lib.fv_last_error()


def test_halley_step_limit_setting(lib):
    """fv_set_halley_steps keeps the limit in [1, 64] and rejects anything
    else without changing the limit in force (host-side only, no launch)."""
    lib.fv_set_halley_steps.argtypes = [ctypes.c_int]
    assert lib.fv_get_halley_steps() == 8
    try:
        for bad in (0, -1, 65):
            assert lib.fv_set_halley_steps(bad) == -1
            assert lib.fv_get_halley_steps() == 8
        for good in (1, 2, 64):
            assert lib.fv_set_halley_steps(good) == 0
            assert lib.fv_get_halley_steps() == good
    finally:
        assert lib.fv_set_halley_steps(8) == 0


def test_kernel_code_hash_ignores_comments_only():
    """The hash that ties the bench's stored counter figures to the kernel
    sources changes with the code, not with comments or layout (string
    literals are kept verbatim, including a // inside one)."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    a = 'int f(int x) {\n  return x + 1;  // one\n}\nconst char* p = "a // b";\n'
    b = '/* header */\nint f(int x)\n{ return x + 1; }\n// trailing\nconst char* p = "a // b";'
    c = 'int f(int x) {\n  return x + 2;\n}\nconst char* p = "a // b";\n'
    d = 'int f(int x) {\n  return x + 1;\n}\nconst char* p = "a /* b";\n'
    ca = bench._code_only(a)
    assert ca == bench._code_only(b)
    assert ca != bench._code_only(c)
    assert ca != bench._code_only(d)
    assert '"a // b"' in ca
    assert len(bench.kernel_source_sha256()) == 64
