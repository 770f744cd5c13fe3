"""Host-side checks of the C ABI (no GPU): the library loads and exports
every function the public headers declare."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+(gcm_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("gcm_ctx_create", "gcm_ctx_destroy", "gcm_last_error", "gcm_encrypt", "gcm_decrypt_verify",
                 "gcm_key_register", "gcm_key_release", "gcm_encrypt_async", "gcm_decrypt_verify_async",
                 "gcm_ctr_xcrypt", "gcm_ctr_async", "gcm_gmac", "gcm_encrypt_host", "gcm_decrypt_verify_host",
                 "gcm_set_pipeline", "gcm_encrypt_ex", "gcm_decrypt_verify_ex",
                 "gcm_stream_begin", "gcm_stream_update", "gcm_stream_final", "gcm_stream_destroy",
                 "gcm_fits_encrypt", "gcm_fits_decrypt", "gcm_fits_free", "gcm_fits_nonce",
                 "gcm_siv_workspace_size", "gcm_siv_encrypt_async", "gcm_siv_decrypt_verify_async"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2602_23067_amd import gcm

    if not os.path.exists(gcm.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(gcm.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2602_23067_amd import gcm

    monkeypatch.setattr(gcm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gcm, "_lib", None)
    with pytest.raises(ImportError):
        gcm.load()


def test_last_error_is_a_string_before_any_call():
    from paper_2602_23067_amd import gcm

    if not os.path.exists(gcm.LIB_PATH):
        pytest.skip("library not built")
    assert isinstance(gcm.load().gcm_last_error(), bytes)


def test_every_entry_point_contains_exceptions():
    """No C++ exception may cross the C ABI: every multi-line extern "C"
    function in the runtime runs its body between GCM_ABI_TRY and a
    GCM_ABI_CATCH form (one-line accessors excepted)."""
    src_dir = os.path.join(ROOT, "paper_2602_23067_amd", "csrc")
    checked = 0
    for path in sorted(glob.glob(os.path.join(src_dir, "*.cpp"))):
        lines = open(path).read().split("\n")
        for i, line in enumerate(lines):
            if not line.startswith('extern "C"') or line.rstrip().endswith("}"):
                continue
            j = i
            while lines[j] != "{":
                j += 1
            k = j
            while lines[k] != "}":
                k += 1
            name = re.search(r"(gcm_\w+)\(", line).group(1)
            assert lines[j + 1].strip() == "GCM_ABI_TRY", (path, name)
            assert lines[k - 1].strip().startswith("GCM_ABI_CATCH"), (path, name)
            checked += 1
    assert checked >= 40


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as strict C99 and as C++ (no torch or
    HIP types in any signature), and a C program can take every entry
    point's address through it."""
    import subprocess
    hdr = os.path.join(ROOT, "include", "gcm_mi355.h")
    names = sorted(_declared())
    prog = tmp_path / "uses_header.c"
    prog.write_text('#include "gcm_mi355.h"\n'
                    "typedef void (*fn)(void);\n"
                    "const fn entry_points[] = {\n" + ",\n".join(f"    (fn)&{n}" for n in names) + "\n};\n")
    inc = os.path.dirname(hdr)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                    "-I", inc, str(prog)], check=True)
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", hdr], check=True)


def test_noalloc_scratch_size_matches_the_header():
    """The binding's constant for the fixed device scratch is the header's."""
    from paper_2602_23067_amd import gcm

    text = open(os.path.join(ROOT, "include", "gcm_mi355.h")).read()
    m = re.search(r"#define GCM_NOALLOC_SCRATCH_BYTES \(\(1ull << (\d+)\) \+ (\d+)\)", text)
    assert m, "GCM_NOALLOC_SCRATCH_BYTES not found"
    assert gcm.NOALLOC_SCRATCH_BYTES == (1 << int(m.group(1))) + int(m.group(2))
