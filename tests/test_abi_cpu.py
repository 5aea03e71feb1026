"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/lloid.h declares, and reports a missing device as
an error code rather than crashing.  The host planning arithmetic that the
kernels rely on is checked against the oracle's range rule."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lloid.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lloid_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("lloid_bank_create", "lloid_filter", "lloid_ctx_create", "lloid_bank_sigma2"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2410_16416_amd import lloid
    lib = ctypes.CDLL(lloid.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert set(lloid.exported_symbols()) <= set(declared_functions())


def test_binding_constants_match_the_header_macros():
    """The binding's copies of the header's size and count macros."""
    from paper_2410_16416_amd import lloid
    text = open(HEADER).read()
    macros = {m.group(1): m.group(2) for m in re.finditer(r"#define (LLOID_[A-Z0-9_]+) (.+)", text)}
    assert eval(macros["LLOID_NOALLOC_SCRATCH_BYTES"].replace("ll", "")) == lloid.NOALLOC_SCRATCH_BYTES
    assert int(macros["LLOID_FIR_VARIANTS"]) == lloid.FIR_VARIANTS
    assert int(macros["LLOID_MIX_VARIANTS"]) == lloid.MIX_VARIANTS


def test_struct_layouts_match_the_c_header(tmp_path):
    """Compile a C probe of the header with gcc and compare sizes and offsets
    with the ctypes mirrors the binding passes through the boundary."""
    from paper_2410_16416_amd import lloid
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "lloid.h"
#define P(T, F) printf(#T "." #F " %zu\\n", offsetof(T, F));
int main(void) {
  printf("lloid_slice %zu\\n", sizeof(lloid_slice));
  printf("lloid_bank_desc %zu\\n", sizeof(lloid_bank_desc));
  printf("lloid_bank_info %zu\\n", sizeof(lloid_bank_info));
  printf("lloid_trigger %zu\\n", sizeof(lloid_trigger));
  printf("lloid_trigger_opts %zu\\n", sizeof(lloid_trigger_opts));
  printf("lloid_peaks %zu\\n", sizeof(lloid_peaks));
  printf("lloid_stream_opts %zu\\n", sizeof(lloid_stream_opts));
  printf("lloid_stream_stats %zu\\n", sizeof(lloid_stream_stats));
  printf("lloid_coinc %zu\\n", sizeof(lloid_coinc));
  printf("lloid_condition_opts %zu\\n", sizeof(lloid_condition_opts));
  printf("lloid_tune_result %zu\\n", sizeof(lloid_tune_result));
  P(lloid_condition_opts, gate_threshold) P(lloid_condition_opts, psd)
  P(lloid_coinc, bank) P(lloid_coinc, template_id) P(lloid_coinc, snr_net) P(lloid_coinc, dt)
  P(lloid_stream_opts, use_graph) P(lloid_stream_opts, hbm_budget) P(lloid_stream_opts, trig)
  P(lloid_stream_stats, bytes_in_use) P(lloid_stream_stats, graph_replays)
  P(lloid_slice, start_tap) P(lloid_slice, basis) P(lloid_slice, mixing)
  P(lloid_trigger, window) P(lloid_trigger, sample) P(lloid_trigger, snr) P(lloid_trigger, phase)
  P(lloid_trigger, snr_interp) P(lloid_trigger, dt) P(lloid_trigger, xi2)
  P(lloid_bank_desc, slices) P(lloid_bank_desc, autocorr_half) P(lloid_bank_desc, autocorr)
  P(lloid_bank_info, device_bytes)
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    mirror = {"lloid_slice": lloid.lloid_slice, "lloid_bank_desc": lloid.lloid_bank_desc,
              "lloid_bank_info": lloid.lloid_bank_info, "lloid_trigger_opts": lloid.lloid_trigger_opts,
              "lloid_peaks": lloid.lloid_peaks, "lloid_stream_opts": lloid.lloid_stream_opts,
              "lloid_stream_stats": lloid.lloid_stream_stats, "lloid_condition_opts": lloid.lloid_condition_opts}
    for name, cls in mirror.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
    assert int(got["lloid_trigger"]) == lloid.TRIGGER_DTYPE.itemsize
    assert int(got["lloid_coinc"]) == lloid.COINC_DTYPE.itemsize
    assert int(got["lloid_tune_result"]) == lloid.TUNE_DTYPE.itemsize
    from workloads.triggers import TRIGGER_DTYPE as synthetic
    assert synthetic == lloid.TRIGGER_DTYPE
    for f in ("bank", "template_id", "snr_net", "dt"):
        assert int(got[f"lloid_coinc.{f}"]) == lloid.COINC_DTYPE.fields[f][1], f
    for f in ("xi2", "window", "sample", "snr", "phase", "snr_interp", "dt"):
        assert int(got[f"lloid_trigger.{f}"]) == lloid.TRIGGER_DTYPE.fields[f][1]
    for f in ("start_tap", "basis", "mixing"):
        assert int(got[f"lloid_slice.{f}"]) == getattr(lloid.lloid_slice, f).offset
    for f in ("slices", "autocorr_half", "autocorr"):
        assert int(got[f"lloid_bank_desc.{f}"]) == getattr(lloid.lloid_bank_desc, f).offset, f
    assert int(got["lloid_bank_info.device_bytes"]) == lloid.lloid_bank_info.device_bytes.offset
    for f in ("use_graph", "hbm_budget", "trig"):
        assert int(got[f"lloid_stream_opts.{f}"]) == getattr(lloid.lloid_stream_opts, f).offset, f
    for f in ("gate_threshold", "psd"):
        assert int(got[f"lloid_condition_opts.{f}"]) == getattr(lloid.lloid_condition_opts, f).offset, f
    for f in ("bytes_in_use", "graph_replays"):
        assert int(got[f"lloid_stream_stats.{f}"]) == getattr(lloid.lloid_stream_stats, f).offset, f


def test_missing_device_is_an_error_code():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2410_16416_amd import lloid
    with pytest.raises(lloid.LloidError) as ei:
        lloid.lloid_ctx_create(0)
    assert ei.value.status == lloid.LLOID_EDEVICE
    assert "not available" in str(ei.value)


def test_level_ranges_rule():
    """The interpolation halo rule the host plan uses (ceil((lo-32)/2),
    floor((hi-1+32)/2)+1) reproduces the oracle's brute-force support."""
    need = oracle.level_ranges(0, 1000, 5)
    assert need[1] == (-16, 516)
    for (lo, hi), (lo2, hi2) in zip(need[:-1], need[1:]):
        # every j with |n - 2j| <= 32 for some n in [lo, hi) lies in [lo2, hi2)
        js = {j for n in (lo, hi - 1) for j in range((n - 32 + 1) // 2 - 1, (n + 32) // 2 + 2)
              if abs(n - 2 * j) <= 32}
        assert min(js) == lo2 and max(js) == hi2 - 1
