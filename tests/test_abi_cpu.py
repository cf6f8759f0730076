"""The C ABI library without a GPU: it loads, exports every symbol that
include/gsm.h declares, and its host-side argument checks answer correctly
(none of these calls reaches the device)."""
import ctypes
import os
import re

import pytest

from paper_2003_01527_amd import gsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fname in os.listdir(os.path.join(ROOT, "include")):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gsm_\w+)\s*\(", text):
            if not m.group(1).endswith("_fn"):
                names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("gsm_graph_create", "gsm_query_create", "gsm_match", "gsm_match_batch",
                     "gsm_filter", "gsm_query_plan"):
        assert required in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_declared_symbol(name):
    lib = ctypes.CDLL(gsm.library_path())
    assert hasattr(lib, name), name


def test_status_strings():
    lib = gsm._load()
    assert lib.gsm_status_str(0) == b"ok"
    assert lib.gsm_status_str(7) == b"output truncated"


def test_struct_sizes_match_header():
    # gsm_match_opts: u32 + pad, u64, 4 x i32, ptr, i32, 2 x u32, 3 ptrs, 3 x i32 (+pad)
    assert ctypes.sizeof(gsm.MatchOpts) == 112
    assert ctypes.sizeof(gsm.Stats) == 8 + 8 + 3 * 16 * 8 + 4 * 8 + 2 * 8 + 8
    o = gsm.make_opts()
    assert o.struct_size == ctypes.sizeof(gsm.MatchOpts)
    assert o.filter_rounds == 1 and o.use_degree == 1 and o.use_ne == 1 and o.root_qvertex == -1


@pytest.mark.parametrize("q,edges,labels", [
    (0, [], None),                        # empty query
    (17, [(i, i + 1) for i in range(16)], None),  # too large
    (3, [(0, 1)], None),                  # disconnected
    (3, [(0, 1), (1, 1), (1, 2)], None),  # self-loop
    (3, [(0, 1), (1, 0), (1, 2)], None),  # duplicate edge
    (2, [(0, 2)], None),                  # out of range
    (2, [(0, 1)], [0, -1]),               # negative label
])
def test_query_create_rejects(q, edges, labels):
    with pytest.raises(gsm.GsmError) as ei:
        gsm.Query(q, edges, labels)
    assert ei.value.status == 3


def test_query_create_accepts_single_vertex_and_k16():
    gsm.Query(1, [], None).close()
    gsm.Query(16, [(a, b) for a in range(16) for b in range(a + 1, 16)], None).close()


def test_graph_create_rejects_bad_arguments_before_device():
    lib = gsm._load()
    h = ctypes.c_void_p()
    assert lib.gsm_graph_create(-1, None, None, None, 0, ctypes.byref(h)) == 1
    assert lib.gsm_graph_create(4, None, None, None, 0, ctypes.byref(h)) == 1
    assert lib.gsm_graph_create(4, None, None, None, 0, None) == 1
    assert lib.gsm_last_error() != b""


def test_match_rejects_null_handles():
    lib = gsm._load()
    cnt = ctypes.c_uint64()
    assert lib.gsm_match(None, None, None, ctypes.byref(cnt), None, 0, None) == 1
    assert lib.gsm_match_batch(None, 0, None, None, None) == 1


def test_binding_flags_match_header():
    text = open(os.path.join(ROOT, "include", "gsm.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(GSM_\w+)\s+(\d+)u?", text)}
    assert defs["GSM_GRAPH_VALIDATE"] == gsm.GRAPH_VALIDATE
    assert defs["GSM_GRAPH_DEVICE_PTRS"] == gsm.GRAPH_DEVICE_PTRS
    assert defs["GSM_GRAPH_STRIP"] == gsm.GRAPH_STRIP
    assert defs["GSM_GRAPH_NO_HUB_BITMAPS"] == gsm.GRAPH_NO_HUB_BITMAPS
    assert defs["GSM_GRAPH_DEGREE_ORDER"] == gsm.GRAPH_DEGREE_ORDER
    assert defs["GSM_MATCH_NO_OUTPUT_STAGING"] == gsm.FLAG_NO_OUTPUT_STAGING
    assert defs["GSM_MATCH_SORT_ROWS"] == gsm.FLAG_SORT_ROWS
    assert defs["GSM_MATCH_LOOKAHEAD"] == gsm.FLAG_LOOKAHEAD
    assert defs["GSM_MATCH_UNIQUE"] == gsm.FLAG_UNIQUE
    assert defs["GSM_MATCH_INDUCED"] == gsm.FLAG_INDUCED
    assert defs["GSM_MATCH_PACK_FRONTIER"] == gsm.FLAG_PACK_FRONTIER
    assert defs["GSM_MATCH_LOOKAHEAD2"] == gsm.FLAG_LOOKAHEAD2
    assert defs["GSM_MATCH_HOST_LEVELS"] == gsm.FLAG_HOST_LEVELS
    assert defs["GSM_MATCH_NO_GRAPH"] == gsm.FLAG_NO_GRAPH
    assert defs["GSM_MAX_QUERY_VERTICES"] == 16
    flags = gsm.make_opts(sort_rows=True, lookahead=True, unique=True, induced=True, stage_output=False).flags
    assert flags == (gsm.FLAG_SORT_ROWS | gsm.FLAG_LOOKAHEAD | gsm.FLAG_UNIQUE | gsm.FLAG_INDUCED
                     | gsm.FLAG_NO_OUTPUT_STAGING)
