"""C-ABI library: loads, exports every declared symbol, and validates arguments (CPU only).

No call here launches GPU work: only size queries and argument checks that fail
before anything is enqueued.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\**\s+\**\s*([a-z_]+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def binding():
    from paper_2011_11120_amd import mdc
    return mdc


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("mdc_query_sizes", "mdc_create", "mdc_forward", "mdc_adjoint", "mdc_destroy",
                 "lsqr_solve", "mch_forward", "mch_adjoint"):
        assert name in fns


def test_library_exports_every_declared_symbol(binding):
    lib = C.CDLL(binding.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert missing == []
    assert set(declared_functions()) <= set(binding.EXPORTS)


def test_resident_size_matches_table1_kernel_sizes(binding):
    # Table 1: kernel of 300 frequencies x n x n complex64 (Full 230 GB ... Sub8 3 GB)
    for n, gb in ((9801, 230), (4901, 57), (2451, 14), (1126, 3)):
        d = binding.mdc_desc(1024, 300, n, n, 1, binding.MDC_FP32)
        res, work = binding.mdc_query_sizes(d)
        assert abs(300 * n * n * 8 / 1e9 - gb) < 1.0
        # rows padded to a multiple of 4 columns, plus small tables
        assert 300 * n * n * 8 <= res < 300 * n * (n + 4) * 8 + 64 * 1024
        d16 = binding.mdc_desc(1024, 300, n, n, 1, binding.MDC_FP16S)
        assert binding.mdc_query_sizes(d16)[0] < res * 0.51


@pytest.mark.parametrize("bad,code", [
    (dict(nt=100), -7), (dict(nt=4096), -7), (dict(nfmax=0), -1), (dict(nfmax=514), -1),
    (dict(ns=0), -1), (dict(nr=0), -1), (dict(max_cols=0), -1), (dict(prec=9), -1),
])
def test_invalid_descriptors_are_rejected(binding, bad, code):
    kw = dict(nt=1024, nfmax=300, ns=64, nr=64, max_cols=4, prec=0)
    kw.update(bad)
    d = binding.mdc_desc(kw["nt"], kw["nfmax"], kw["ns"], kw["nr"], kw["max_cols"], kw["prec"])
    with pytest.raises(binding.MdcError) as ei:
        binding.mdc_query_sizes(d)
    assert ei.value.status == code
    assert binding.mdc_last_error()


def test_null_handles_are_rejected(binding):
    lib = binding._lib
    assert lib.mdc_forward(None, None, None, 1, None) == binding.MDC_EINVAL
    assert lib.mdc_destroy(None) == binding.MDC_OK
    assert lib.lsqr_query_sizes(None, None, None) == binding.MDC_EINVAL
