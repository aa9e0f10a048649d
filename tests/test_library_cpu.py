"""The C-ABI library loads without a GPU and exports every symbol that
include/rplu.h declares; no compute calls are made here."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rplu.h")
LIB = os.path.join(ROOT, "paper_2601_22344_amd", "librplu.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rplu_[a-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = _declared()
    for required in ("rplu_dense", "rplu_cauchy", "rplu_batched", "rplu_server_submit",
                     "rplu_server_poll", "rplu_create", "rplu_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "librplu.so is not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.rplu_status_str.restype = ctypes.c_char_p
    assert lib.rplu_status_str(0) == b"RPLU_OK"
    assert lib.rplu_status_str(-7) == b"RPLU_E_ZERO_PIVOT"


def _header_constants():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body in re.findall(r"enum\s*\w*\s*\{(.*?)\}", src, flags=re.S):
        nxt = 0
        for item in body.split(","):
            item = item.strip()
            if not item:
                continue
            if "=" in item:
                name, expr = (s.strip() for s in item.split("=", 1))
                nxt = eval(re.sub(r"(\d+)u\b", r"\1", expr), {})   # integer literals and <<
            else:
                name = item
            out[name] = nxt
            nxt += 1
    for name, val in re.findall(r"#define\s+(RPLU_[A-Z0-9_]+)\s+(\d+)\s*$", src, flags=re.M):
        out[name] = int(val)
    return out


def test_binding_constants_match_header():
    import paper_2601_22344_amd._binding as B
    consts = _header_constants()
    assert "RPLU_FLAG_SPLIT_SAMPLER" in consts and "RPLU_STOP_STALL" in consts
    assert consts.get("RPLU_FLAG_C2PLU") == 32
    checked = 0
    for name, val in consts.items():
        if hasattr(B, name):
            assert getattr(B, name) == val, name
            checked += 1
    assert checked >= 20


def test_binding_declares_every_signature():
    """Every C function the binding calls has its argument types declared:
    without them ctypes passes a Python int as a 32-bit C int, and an int64_t
    parameter passed on the stack then carries undefined upper bits."""
    import paper_2601_22344_amd._binding as B
    src = open(B.__file__).read()
    called = sorted(set(re.findall(r"\blib\.(rplu_[a-z_]+)\(", src)))
    assert "rplu_cur" in called and "rplu_dense" in called
    missing = [n for n in called if getattr(B.lib, n).argtypes is None]
    assert not missing, missing
