"""The C-ABI library on the CPU: it loads, exports every symbol the public
header declares, and rejects bad arguments before touching the GPU.  The
host-side record layout helpers round-trip.  No compute calls here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1102_0148_amd as corr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "corr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(corr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(corr.LIB_PATH):
        corr_build = __import__("paper_1102_0148_amd.build", fromlist=["build"])
        corr_build.build()
    return corr.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    assert sorted(corr.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("N,K,S", [(1, 256, 16), (513, 256, 16), (44, 100, 16), (44, 64, 16),
                                   (44, 2048, 16), (44, 256, 0), (44, 256, (1 << 24) + 1)])
def test_create_rejects_bad_shapes(lib, N, K, S):
    assert lib.corr_create(N, K, S) is None
    msg = corr.corr_last_error()
    assert msg and ("N=" in msg or "K=" in msg or "n_spectra" in msg)


def test_null_handle_is_rejected(lib):
    assert lib.corr_set_precision(None, 0) == corr.CORR_EINVAL
    assert lib.corr_process(None, None, None) == corr.CORR_EINVAL
    assert lib.corr_read_cps_raw(None, None) == corr.CORR_EINVAL
    assert lib.corr_spectra_bytes(None, 16) == 0
    lib.corr_destroy(None)  # NULL-safe


@pytest.mark.parametrize("prec", [corr.CORR_FP32, corr.CORR_FP16, corr.CORR_INT8])
@pytest.mark.parametrize("N,S", [(5, 7), (44, 33), (70, 9)])
def test_record_layout_round_trip(prec, N, S):
    K = 8
    rng = np.random.default_rng(prec * 100 + N)
    if prec == corr.CORR_INT8:
        spec = rng.integers(-127, 128, (S, N, K, 2)).astype(np.int8)
    else:
        spec = (rng.standard_normal((S, N, K)) + 1j * rng.standard_normal((S, N, K))).astype(np.complex64)
        if prec == corr.CORR_FP16:
            spec = spec.real.astype(np.float16).astype(np.float32) + 1j * spec.imag.astype(np.float16).astype(np.float32)
    buf = corr.spectra_to_records(spec, prec)
    tg = corr.record_times(prec)
    a_pad = corr.a_pad_of(N)
    ntq = ((S + tg - 1) // tg + 15) // 16 * 16
    assert buf.size == K * ntq * a_pad * 16
    back = corr.records_to_spectra(buf, prec, N, K, S)
    np.testing.assert_array_equal(back, spec)
    # one record by hand: channel 3, antenna 2, spectra 0..tg-1 as [re x tg][im x tg]
    dt = {corr.CORR_FP32: np.float32, corr.CORR_FP16: np.float16, corr.CORR_INT8: np.int8}[prec]
    rec = buf.view(dt).reshape(-1, K, 16, a_pad, 2 * tg)[0, 3, 0, 2]
    n = min(tg, S)
    if prec == corr.CORR_INT8:
        np.testing.assert_array_equal(rec[:n], spec[:n, 2, 3, 0])
        np.testing.assert_array_equal(rec[tg:tg + n], spec[:n, 2, 3, 1])
    else:
        np.testing.assert_array_equal(rec[:n].astype(np.float32), spec[:n, 2, 3].real)
        np.testing.assert_array_equal(rec[tg:tg + n].astype(np.float32), spec[:n, 2, 3].imag)


@pytest.mark.parametrize("N,S", [(5, 7), (44, 33), (70, 9)])
def test_int16_record_layout_round_trip(N, S):
    """int16 records: codes within +-32512 round-trip through the base-255
    digit layout [h of re x4][h of im x4][l of re x4][l of im x4], and one
    record checked by hand."""
    K = 8
    rng = np.random.default_rng(1600 + N)
    spec = rng.integers(-32512, 32513, (S, N, K, 2)).astype(np.int16)
    spec[0, 0, 0] = (32512, -32512)
    buf = corr.spectra_to_records(spec, corr.CORR_INT16)
    a_pad = corr.a_pad_of(N)
    ntq = ((S + 3) // 4 + 15) // 16 * 16
    assert buf.size == K * ntq * a_pad * 16
    np.testing.assert_array_equal(corr.records_to_spectra(buf, corr.CORR_INT16, N, K, S), spec)
    rec = buf.view(np.int8).reshape(-1, K, 16, a_pad, 16)[0, 3, 0, 2].astype(np.int32)
    n = min(4, S)
    q = spec[:n, 2, 3].astype(np.int32)  # [t][re, im]
    np.testing.assert_array_equal(255 * rec[0:n] + rec[8:8 + n], q[:, 0])
    np.testing.assert_array_equal(255 * rec[4:4 + n] + rec[12:12 + n], q[:, 1])
    assert np.abs(rec).max() <= 127


def test_binding_constants_match_header():
    text = open(HEADER).read()
    for name in ("CORR_MAX_ANTENNAS", "CORR_MAX_CHANNELS", "CORR_CALIB_SPECTRA", "CORR_FRAME_HEADER_BYTES"):
        m = re.search(rf"#define {name} (\d+)", text)
        if m and hasattr(corr, name):
            assert getattr(corr, name) == int(m.group(1)), name
    assert corr.CORR_MAX_ANTENNAS == int(re.search(r"#define CORR_MAX_ANTENNAS (\d+)", text).group(1))
    assert corr.CORR_MAX_CHANNELS == int(re.search(r"#define CORR_MAX_CHANNELS (\d+)", text).group(1))



def test_noalloc_rejects_bad_arguments_before_any_hip_call(lib):
    """The no-allocation entry point checks shape, precision, pointers and
    its scratch budget on the host (no GPU here)."""
    ok_ptr = 1 << 20                     # aligned, never dereferenced
    cases = [
        (1, 256, 16, corr.CORR_FP32, ok_ptr, ok_ptr, None),          # N too small
        (44, 100, 16, corr.CORR_FP32, ok_ptr, ok_ptr, None),         # K not a power of two
        (44, 256, 16, 9, ok_ptr, ok_ptr, None),                      # unknown precision
        (44, 256, 70000, corr.CORR_INT8, ok_ptr, ok_ptr, ok_ptr),    # int8 over 65536 spectra
        (44, 256, 16, corr.CORR_FP32, None, ok_ptr, None),           # no input
        (44, 256, 16, corr.CORR_FP32, ok_ptr + 1, ok_ptr, None),     # misaligned input
        (44, 256, 16, corr.CORR_FP32, ok_ptr, ok_ptr + 8, None),     # misaligned output
        (44, 256, 16, corr.CORR_INT8, ok_ptr, ok_ptr, None),         # int8 without scales
        (256, 512, 64, corr.CORR_FP32, ok_ptr, ok_ptr, None),        # does not fit the scratch
        (512, 1024, 45, corr.CORR_INT16, ok_ptr, ok_ptr, ok_ptr),    # does not fit the scratch
    ]
    for args in cases:
        assert lib.corr_process_noalloc(*args, None) == corr.CORR_EINVAL, args
        assert corr.corr_last_error()
    lib.corr_process_noalloc(256, 512, 64, corr.CORR_FP32, ok_ptr, ok_ptr, None, None)
    assert "bytes of scratch" in corr.corr_last_error()
