"""The C-ABI library loads, exports every symbol include/wmd.h declares, and
rejects bad arguments on the host before any device work.  No GPU needed:
every call below fails validation before it would touch the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2107_06433_amd import wmd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="wmd.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wmd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = wmd.load_library()
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert headers == ["wmd.h", "wmd_bench.h"]
    declared = header_functions("wmd.h")
    assert declared, "no declarations parsed"
    assert sorted(wmd.EXPORTS) == declared
    assert sorted(wmd.BENCH_EXPORTS) == header_functions("wmd_bench.h")
    for name in declared + wmd.BENCH_EXPORTS:
        assert hasattr(lib, name), name


def test_measurement_kernels_reject_bad_arguments():
    lib = wmd.load_library()
    assert lib.wmd_bench_stream(None, None, 1024, 0, 1, None, None) == 1
    assert lib.wmd_bench_stream(1, None, 1000, 1, 1, None, None) == 1   # copy without dst; bytes not /16
    assert lib.wmd_bench_gather(1, 6, 1, 10, 1, 1, None) == 1          # S not a multiple of 4
    assert lib.wmd_bench_gather(1, 516, 1, 10, 1, 1, None) == 1        # S past 512
    assert lib.wmd_bench_valu(1, 1, 1, 7, None) == 1                    # unknown mode
    assert lib.wmd_bench_tiles(1, 10, 100, 1, None) == 1                 # row bytes not a multiple of 64


def test_ctypes_structs_match_header_layout():
    # sizes implied by the C declarations on LP64
    assert ctypes.sizeof(wmd.CorpusDesc) == 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(wmd.QueryDesc) == 8 + 8 + 8 + 8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 8 + 8
    assert ctypes.sizeof(wmd.CorpusInfo) == 3 * 8 + 2 * 4 + 8 + 8 + 8 + 16 * 8 + 16 * 4


def test_workspace_sizes():
    lib = wmd.load_library()
    assert lib.wmd_corpus_workspace_bytes(0, 300, 10, 10) == 0
    assert lib.wmd_corpus_workspace_bytes(100, 0, 10, 10) == 0
    assert lib.wmd_corpus_workspace_bytes(100, 5000, 10, 10) == 0
    assert lib.wmd_corpus_workspace_bytes(100, 300, 0, 10) == 0
    a = lib.wmd_corpus_workspace_bytes(100_000, 300, 5_000, 300_000)
    # at least the f32 and bf16 embedding copies (padded to 320) and the per-entry arrays
    assert a >= 100_000 * 320 * 6 + 300_000 * 8
    assert a % 256 == 0
    qp = np.array([0, 5], dtype=np.int64)
    assert lib.wmd_query_workspace_bytes(None, 1, qp.ctypes.data, 0) == 0


def test_host_argument_errors():
    lib = wmd.load_library()
    out = ctypes.c_void_p()
    assert lib.wmd_create_corpus(None, None, ctypes.byref(out)) == 1
    assert b"NULL" in lib.wmd_last_error()
    desc = wmd.CorpusDesc(V=0, d=3, emb=1, N=1, nnz=0, doc_ptr=1, word_ids=1, weights=1,
                          compact_vocab=1, workspace=1, workspace_bytes=1 << 30)
    assert lib.wmd_create_corpus(ctypes.byref(desc), None, ctypes.byref(out)) == 1
    desc.V, desc.d = 10, 5000
    assert lib.wmd_create_corpus(ctypes.byref(desc), None, ctypes.byref(out)) == 1
    desc.d, desc.emb = 5, None
    assert lib.wmd_create_corpus(ctypes.byref(desc), None, ctypes.byref(out)) == 1
    desc.emb, desc.workspace_bytes = 1, 16
    assert lib.wmd_create_corpus(ctypes.byref(desc), None, ctypes.byref(out)) == 2
    assert b"workspace" in lib.wmd_last_error()
    desc.workspace_bytes = 1 << 30  # large enough, but the pointer is not 256-byte aligned
    assert lib.wmd_create_corpus(ctypes.byref(desc), None, ctypes.byref(out)) == 1
    assert b"aligned" in lib.wmd_last_error()
    assert out.value is None
    q = wmd.QueryDesc(B=1, q_ptr_host=None, q_ptr=1, q_ids=1, q_weights=1, lam=10.0,
                      max_iter=15, cdist=0, schedule=0)
    assert lib.wmd_query(None, ctypes.byref(q), 1, 1, 1, None) == 1
    assert lib.wmd_query_errors(None, 1, None, None) == 1
    assert lib.wmd_destroy(None) == 0
    assert lib.wmd_last_error() == b""


def test_query_descriptor_validation_messages():
    lib = wmd.load_library()
    # a non-NULL but fake corpus pointer is never dereferenced before the
    # descriptor checks fail
    fake = ctypes.c_void_p(1)
    for field, value in [("lam", 0.0), ("lam", float("nan")), ("max_iter", -1), ("cdist", 7), ("schedule", 9),
                         ("tol", -1.0), ("tol", float("inf"))]:
        q = wmd.QueryDesc(B=1, q_ptr_host=1, q_ptr=1, q_ids=1, q_weights=1, lam=10.0,
                          max_iter=15, cdist=0, schedule=0)
        setattr(q, field, value)
        assert lib.wmd_query(fake, ctypes.byref(q), 1, 1, 1, None) == 1, field
