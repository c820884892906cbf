"""The C ABI library loads and exports every function include/hetm.h
declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hetm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w ]+\*?\s*\b(hetm_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def hm():
    from paper_1905_00661_amd import hetm
    if not os.path.exists(hetm.LIB_PATH):
        pytest.fail("libhetm.so not built: run __graft_entry__.build()")
    return hetm


def test_exports_every_declared_symbol(hm):
    L = hm.lib()
    names = declared()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hm.EXPORTS)


def test_strerror_and_null_handling(hm):
    L = hm.lib()
    assert L.hetm_strerror(0) == b"ok"
    assert L.hetm_strerror(hm.HETM_EORDER) == b"timestamp order violated"
    assert L.hetm_submit_batch(None, 1, None, 0, None, None) == hm.HETM_EINVAL
    assert L.hetm_round(None, None, None) == hm.HETM_EINVAL
    assert L.hetm_sync(None) == hm.HETM_EINVAL
    assert L.hetm_read_words_noalloc(None, 0, 0, None) == hm.HETM_EINVAL
    assert L.hetm_round_begin(None, None) == hm.HETM_EINVAL
    assert L.hetm_round_push(None, None, 0, None) == hm.HETM_EINVAL
    assert L.hetm_round_add(None, 1, None, 0, None, None) == hm.HETM_EINVAL
    assert L.hetm_round_end(None, None) == hm.HETM_EINVAL
    assert L.hetm_round_submit(None, None) == hm.HETM_EINVAL
    assert L.hetm_round_collect(None, None) == hm.HETM_EINVAL


@pytest.mark.parametrize("field,value", [("n_words", 0), ("word_bytes", 2), ("granule_words", 0),
                                         ("lock_stripe_words", 3), ("max_txn_ops", 65), ("mode", 7),
                                         ("log_capacity", 0), ("log_capacity", (1 << 29) + 1)])
def test_config_rejected_before_touching_a_device(hm, field, value):
    cfg = hm.hetm_config(n_words=1024, word_bytes=4, granule_words=1, lock_stripe_words=1, max_txn_ops=8,
                         batch_capacity=16, log_capacity=16, mode=0, device=0, stream=None)
    setattr(cfg, field, value)
    out = ctypes.c_void_p()
    assert hm.lib().hetm_alloc_stmr(ctypes.byref(cfg), None, ctypes.byref(out)) == hm.HETM_EINVAL
    assert out.value is None


def test_struct_layouts_match_header(hm, tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a C
    compiler makes of include/hetm.h."""
    structs = {n: getattr(hm, n) for n in ["hetm_config", "hetm_oplist_desc", "hetm_transfer_desc",
                                           "hetm_cache_desc", "hetm_round_args", "hetm_round_result",
                                           "hetm_stats", "hetm_serve_spec", "hetm_serve_report"]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hetm.h"', "int main(void) {"]
    for n, cls in structs.items():
        lines.append(f'printf("{n} sizeof %zu\\n", sizeof({n}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for n, cls in structs.items():
        assert got[(n, "sizeof")] == ctypes.sizeof(cls), n
        for f, _ in cls._fields_:
            assert got[(n, f)] == getattr(cls, f).offset, (n, f)
