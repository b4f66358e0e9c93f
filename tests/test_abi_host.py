"""The C ABI on a host without a GPU: the library loads, exports every symbol
the header declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2003_09133_amd import _abi
from paper_2003_09133_amd._abi import GatherConfig, Problem, Shape

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lfbp.h")
GOOD = Shape(15, 15, 3, 3, 3)
P1, P2 = 0x10000, 0x20000000          # fake device addresses, never dereferenced


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^LFBP_API\s+[\w\s\*]+?\b(lfbp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("lfbp_compute_Ht", "lfbp_compute_Ht_batched", "lfbp_forward", "lfbp_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(declared_functions()) <= exported
    # only the ABI is exported
    assert {s for s in exported if s.startswith("lfbp")} == set(declared_functions())


def test_status_strings():
    L = _abi.lib()
    for code in range(0, -10, -1):
        assert L.lfbp_status_string(code) and b"unknown" not in L.lfbp_status_string(code)
    assert b"unknown" in L.lfbp_status_string(-99)
    assert L.lfbp_version().startswith(b"lfbp")


def call(H=P1, Ht=P2, shape=GOOD, dt=_abi.F32):
    return _abi.lib().lfbp_compute_Ht(H, Ht, shape, dt, None)


@pytest.mark.parametrize("shape", [Shape(0, 15, 3, 3, 3), Shape(15, 15, 3, 3, 0), Shape(14, 15, 3, 3, 3),
                                   Shape(15, 16, 3, 3, 3), Shape(15, 15, 4, 3, 3), Shape(15, 15, 3, 2, 3),
                                   Shape(-1, 15, 3, 3, 3), Shape(65537, 65537, 1, 1, 1),
                                   Shape(1, 1, 3, 3, 1 << 28), Shape(1 << 40, 1, 1, 1, 1)])
def test_bad_shapes(shape):
    assert call(shape=shape) == _abi.ESHAPE


def test_null_dtype_alias_align():
    assert call(H=None) == _abi.EINVAL
    assert call(Ht=None) == _abi.EINVAL
    assert call(dt=7) == _abi.EDTYPE
    assert call(Ht=P1) == _abi.EALIAS
    nbytes = 15 * 15 * 3 * 3 * 3 * 4
    assert call(Ht=P1 + nbytes - 4) == _abi.EALIAS
    assert call(H=P1 + 2) == _abi.EALIGN
    assert call(Ht=P2 + 1, dt=_abi.F16) == _abi.EALIGN


def test_bad_config_fields():
    L = _abi.lib()
    for field, val in [("variant", 4), ("block_threads", 96), ("block_threads", 1024),
                       ("rows_in_flight", 3), ("tile_bytes", 70000), ("vec_per_thread", 3),
                       ("vec_per_thread", 16), ("nontemporal", 3), ("persistent", 3), ("grid", -1),
                       ("waves_per_eu", 9), ("waves_per_eu", -1), ("schedule", 3), ("schedule", -1)]:
        c = GatherConfig()
        setattr(c, field, val)
        assert L.lfbp_compute_Ht_config(P1, P2, GOOD, _abi.F32, ctypes.byref(c), None) == _abi.EINVAL, field


def test_default_config_resolves_every_field():
    L = _abi.lib()
    for shape, dt in [(GOOD, _abi.F32), (Shape(165, 165, 15, 15, 21), _abi.F32),
                      (Shape(345, 345, 15, 15, 51), _abi.F16), (Shape(181, 181, 95, 55, 11), _abi.F32),
                      (Shape(3, 3, 1, 1, 40000), _abi.F32)]:
        c = GatherConfig()
        assert L.lfbp_default_config(shape, dt, ctypes.byref(c)) == _abi.OK
        d = c.as_dict()
        assert all(v > 0 for v in d.values()), d
        assert d["variant"] in (_abi.GATHER_DIRECT, _abi.GATHER_STAGED, _abi.GATHER_WIDE)
    c = GatherConfig()
    assert L.lfbp_default_config(Shape(4, 3, 3, 3, 3), _abi.F32, ctypes.byref(c)) == _abi.ESHAPE
    assert L.lfbp_default_config(GOOD, 9, ctypes.byref(c)) == _abi.EDTYPE
    assert L.lfbp_default_config(GOOD, _abi.F32, None) == _abi.EINVAL


def batch(*probs):
    return (Problem * len(probs))(*probs)


def test_batched_validation_before_launch():
    L = _abi.lib()
    ok = Problem(P1, P2, GOOD)
    assert L.lfbp_compute_Ht_batched(None, 1, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_batched(batch(ok), 0, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_batched(batch(ok), 1, 5, None) == _abi.EDTYPE
    bad_shape = Problem(P1 + 0x100000, P2 + 0x100000, Shape(15, 15, 2, 3, 3))
    assert L.lfbp_compute_Ht_batched(batch(ok, bad_shape), 2, _abi.F32, None) == _abi.ESHAPE
    null = Problem(None, P2 + 0x100000, GOOD)
    assert L.lfbp_compute_Ht_batched(batch(ok, null), 2, _abi.F32, None) == _abi.EINVAL
    # output of one problem overlapping the input of another
    cross = Problem(P2 + 0x100000, P1 + 64, GOOD)
    assert L.lfbp_compute_Ht_batched(batch(ok, cross), 2, _abi.F32, None) == _abi.EALIAS
    # two outputs overlapping
    twin = Problem(P1 + 0x100000, P2 + 8, GOOD)
    assert L.lfbp_compute_Ht_batched(batch(ok, twin), 2, _abi.F32, None) == _abi.EALIAS
    assert L.lfbp_compute_Ht_batched_config(batch(ok), 1, _abi.F32, None, 2, None) == _abi.EINVAL


def test_projector_validation_before_launch():
    L = _abi.lib()
    assert L.lfbp_forward(None, GOOD, P2, 30, 30, P2 + 0x100000, None) == _abi.EINVAL
    assert L.lfbp_forward(P1, GOOD, P2, 0, 30, P2 + 0x100000, None) == _abi.EINVAL
    assert L.lfbp_forward(P1, Shape(15, 14, 3, 3, 3), P2, 30, 30, P2 + 0x100000, None) == _abi.ESHAPE
    assert L.lfbp_forward(P1, GOOD, P2, 30, 30, P2 + 8, None) == _abi.EALIAS
    assert L.lfbp_forward(P1, GOOD, P2, 30, 30, P2 + 0x100002, None) == _abi.EALIGN
    assert L.lfbp_backward(P1, GOOD, P2, 30, 30, P1 + 16, None) == _abi.EALIAS
    assert L.lfbp_backward(P1, GOOD, P2, 1 << 20, 1 << 20, P2 + 0x100000, None) == _abi.ESHAPE


def test_fastdiv_exact(tmp_path):
    """The division-by-invariant-integer helper of the kernels, compiled for
    the host: exact against '/' for edge and random dividends."""
    src = tmp_path / "fd.cpp"
    src.write_text(r'''
#include "lfbp_internal.h"
#include <cstdio>
#include <random>
int main() {
  std::mt19937_64 rng(1);
  const uint32_t ds[] = {1,2,3,5,7,11,15,19,21,51,55,95,165,345,765,4725,11475,65535,65536,1u<<20,(1u<<31)-1,1u<<31,0xffffffffu};
  for (uint32_t d : ds) {
    lfbp::FastDiv f = lfbp::make_fastdiv(d);
    for (int i = 0; i < 200000; ++i) {
      uint32_t n = (i < 1000) ? uint32_t(i) : (i < 2000 ? 0xffffffffu - uint32_t(i - 1000) : uint32_t(rng()));
      if (lfbp::fdiv(n, f) != n / d) { std::printf("FAIL %u %u\n", n, d); return 1; }
      uint32_t m = d * (n / d);  // multiples and their neighbours
      if (lfbp::fdiv(m, f) != m / d || (m && lfbp::fdiv(m - 1, f) != (m - 1) / d)) { std::printf("FAIL m %u %u\n", m, d); return 1; }
    }
  }
  std::printf("ok\n");
  return 0;
}
''')
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{ROOT}/include", f"-I{ROOT}/paper_2003_09133_amd/csrc",
                    str(src), "-o", str(exe)], check=True)
    assert subprocess.run([str(exe)], capture_output=True, text=True).stdout.strip() == "ok"


def test_forward_workspace_validation_before_launch():
    L = _abi.lib()
    shape = Shape(165, 165, 15, 15, 21)
    need = L.lfbp_forward_workspace_size(shape, 600, 600)
    assert need > 179 * 179 * 256 * 24 * 4              # H as records of 22 depths per (shift, class)
    assert L.lfbp_forward_workspace_size(Shape(4, 5, 3, 3, 1), 10, 10) == 0
    assert L.lfbp_forward_workspace_size(shape, 0, 600) == 0
    H, g, f, ws = 0x1000000, 0x40000000, 0x80000000, 0xC0000000
    assert L.lfbp_forward_ws(H, shape, g, 600, 600, f, None, need, None) == _abi.EINVAL
    assert L.lfbp_forward_ws(H, shape, g, 600, 600, f, ws, need - 1, None) == _abi.EINVAL
    assert L.lfbp_forward_ws(H, shape, g, 600, 600, f, ws + 16, need, None) == _abi.EINVAL
    assert L.lfbp_forward_ws(H, shape, g, 600, 600, f, g + 256, need, None) == _abi.EALIAS
    assert L.lfbp_forward_ws(H, shape, g, 600, 600, f, f - 256, need, None) == _abi.EALIAS


def test_backward_workspace_validation_before_launch():
    L = _abi.lib()
    shape = Shape(165, 165, 15, 15, 21)
    need = L.lfbp_backward_workspace_size(shape, 600, 600)
    # A and B records: 24 floats per (stage of 22 (r, r2) pairs, lenslet or column)
    stages = -(-(179 * 179) // 22)
    assert need == (stages * 1600 * 24 * 4 + 255) // 256 * 256 + (stages * 4864 * 24 * 4 + 255) // 256 * 256
    assert L.lfbp_backward_workspace_size(Shape(4, 5, 3, 3, 1), 10, 10) == 0
    assert L.lfbp_backward_workspace_size(shape, 600, 0) == 0
    Ht, f, g, ws = 0x1000000, 0x40000000, 0x80000000, 0x100000000
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, None, need, None) == _abi.EINVAL
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, ws, need - 1, None) == _abi.EINVAL
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, ws + 64, need, None) == _abi.EINVAL
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, f - 512, need, None) == _abi.EALIAS
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, g + 512, need, None) == _abi.EALIAS
    assert L.lfbp_backward_ws(Ht, shape, f, 600, 600, g, Ht + 512, need, None) == _abi.EALIAS
    assert L.lfbp_backward_ws(Ht, Shape(15, 14, 3, 3, 3), f, 30, 30, g, ws, need, None) == _abi.ESHAPE


def test_projector_index_range_limits():
    """Shapes whose operand records would leave the kernels' 32-bit ranges are
    refused before anything runs: (ns+nx-1)(nt+ny-1)nz must stay below 2^31,
    and so must the bytes of one record block (columns, lenslets, or the
    phase-split lenslet grid of g with its zero border)."""
    L = _abi.lib()
    big = Shape(4001, 4001, 101, 101, 150)         # 4101^2 * 150 = 2.5e9 stage-depth products
    assert L.lfbp_forward(P1, big, P2, 30, 30, P2 + 0x100000, None) == _abi.ESHAPE
    assert L.lfbp_backward(P1, big, P2, 30, 30, P2 + 0x100000, None) == _abi.ESHAPE
    assert L.lfbp_forward_workspace_size(big, 30, 30) == 0
    assert L.lfbp_backward_workspace_size(big, 30, 30) == 0
    ok = Shape(4001, 4001, 101, 101, 100)          # 1.7e9 < 2^31
    assert L.lfbp_backward_workspace_size(ok, 30, 30) > 0
    assert L.lfbp_forward_workspace_size(ok, 30, 30) == 0    # 84 M forward stages: a launch-size limit
    border = Shape(20001, 20001, 1, 1, 5)          # g's grid with a 10^4-lenslet zero border: 4e8 records
    assert L.lfbp_forward_workspace_size(border, 30, 30) == 0
    assert L.lfbp_forward_workspace_size(Shape(2001, 2001, 1, 1, 5), 30, 30) > 0


def test_projector_launch_size_limits():
    """Each product is refused when one of its launches would pass 2^24
    workgroups of 256 work-items along a grid dimension (the 32-bit dispatch
    size), and accepted just below: forward B-record stages Kr*Kc*ceil(nz/22),
    the depth transpose of g (R*C/32), the gradient's GEMM tiles."""
    L = _abi.lib()
    fw, bw, gr = L.lfbp_forward_workspace_size, L.lfbp_backward_workspace_size, L.lfbp_grad_psf_workspace_size
    assert fw(Shape(4097, 4097, 1, 1, 1), 8, 8) == 0              # 4097^2 stages >= 2^24
    assert fw(Shape(4095, 4095, 1, 1, 1), 8, 8) > 0               # 4095^2 < 2^24
    assert bw(Shape(4097, 4097, 1, 1, 1), 8, 8) > 0 and gr(Shape(4097, 4097, 1, 1, 1), 8, 8) > 0
    assert fw(Shape(15, 15, 15, 15, 1), 23171, 23171) == 0        # R*C/32 >= 2^24
    assert fw(Shape(15, 15, 15, 15, 1), 23169, 23169) > 0
    assert bw(Shape(15, 15, 15, 15, 1), 23171, 23171) > 0
    assert gr(Shape(4001, 4001, 31, 31, 60), 30, 30) == 0         # 254 k x 226 GEMM tiles
    assert bw(Shape(4001, 4001, 31, 31, 60), 30, 30) > 0
    assert gr(Shape(2001, 2001, 21, 21, 60), 30, 30) > 0          # 64 k x 104
    big = Shape(4097, 4097, 1, 1, 1)
    assert L.lfbp_forward(P1, big, P2, 8, 8, P2 + 0x100000, None) == _abi.ESHAPE
    assert L.lfbp_operator_size(big, 8, 8) == 0 and L.lfbp_rl_workspace_size(big, 8, 8) == 0


def test_batch_overlap_check_against_brute_force():
    """The batch validator's address-ordered sweep against the pairwise
    definition (an output may overlap no input and no other output; inputs
    may overlap).  use_graph = 5 makes every table that passes validation
    return EINVAL before anything could launch."""
    L = _abi.lib()
    rng = np.random.default_rng(7)
    shp = Shape(3, 3, 1, 1, 4)                    # 36 floats = 144 bytes
    nb = 144
    for trial in range(300):
        n = int(rng.integers(1, 9))
        base = 0x100000000
        hs = [base + 16 * int(v) for v in rng.integers(0, 64, n)]
        os_ = [base + 16 * int(v) for v in rng.integers(0, 64, n)]
        probs = (Problem * n)(*[Problem(h, o, shp) for h, o in zip(hs, os_)])
        ov = lambda a, b: a < b + nb and b < a + nb
        bad = any(ov(os_[i], hs[j]) for i in range(n) for j in range(n)) or \
            any(ov(os_[i], os_[j]) for i in range(n) for j in range(i + 1, n))
        st = L.lfbp_compute_Ht_batched_config(probs, n, _abi.F32, None, 5, None)
        assert st == (_abi.EALIAS if bad else _abi.EINVAL), (trial, hs, os_)


def test_rl_validation_before_launch():
    """Every rejected Richardson-Lucy call returns before a launch; a call
    whose only fault is its workspace shows that the in-place form (g_out == g)
    passes the argument checks."""
    L = _abi.lib()
    shape = Shape(15, 15, 3, 3, 3)
    R = C = 30
    vol = 3 * R * C * 4
    H, Ht, f, g, n, o = 0x1000000, 0x2000000, 0x3000000, 0x4000000, 0x5000000, 0x6000000
    need = L.lfbp_rl_workspace_size(shape, R, C)
    assert need >= max(L.lfbp_forward_workspace_size(shape, R, C), L.lfbp_backward_workspace_size(shape, R, C))
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, o, None, need, None) == _abi.EINVAL
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, g, None, need, None) == _abi.EINVAL   # in place: ok
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, g + 4, None, need, None) == _abi.EALIAS
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, n + vol - 4, None, need, None) == _abi.EALIAS
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, Ht + 8, None, need, None) == _abi.EALIAS
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, f, None, need, None) == _abi.EALIAS
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, None, o, None, need, None) == _abi.EINVAL
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, o + 2, None, need, None) == _abi.EALIGN
    assert L.lfbp_rl_step_ws(H, Ht, Shape(15, 14, 3, 3, 3), f, R, C, g, n, o, None, need, None) == _abi.ESHAPE
    assert L.lfbp_rl_step(H, Ht, shape, f, R, C, g, n, g + 4, None) == _abi.EALIAS
    ws = 0x10000000
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, o, g - 256, need, None) == _abi.EALIAS
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, o, ws + 64, need, None) == _abi.EINVAL
    assert L.lfbp_rl_step_ws(H, Ht, shape, f, R, C, g, n, o, ws, need - 1, None) == _abi.EINVAL
    assert L.lfbp_rl_norm_ws(Ht, shape, R, C, Ht + 64, ws, need, None) == _abi.EALIAS
    assert L.lfbp_rl_norm_ws(Ht, shape, R, C, n, None, need, None) == _abi.EINVAL
    assert L.lfbp_rl_workspace_size(Shape(4, 5, 3, 3, 1), 10, 10) == 0


def test_inplace_validation_before_launch():
    L = _abi.lib()
    assert L.lfbp_compute_Ht_inplace(None, GOOD, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_inplace(P1, GOOD, 7, None) == _abi.EDTYPE
    assert L.lfbp_compute_Ht_inplace(P1, Shape(15, 14, 3, 3, 3), _abi.F32, None) == _abi.ESHAPE
    assert L.lfbp_compute_Ht_inplace(P1 + 2, GOOD, _abi.F32, None) == _abi.EALIGN
    # an x-row pair of 2 * 9 * 1000 * 4 bytes does not fit 64 KB of LDS
    assert L.lfbp_compute_Ht_inplace(P1, Shape(3, 3, 3, 9, 1000), _abi.F32, None) == _abi.ESHAPE


def test_grad_psf_validation_before_launch():
    L = _abi.lib()
    shape, R, C = GOOD, 30, 30
    w, g, dH = 0x1000000, 0x2000000, 0x3000000
    need = L.lfbp_grad_psf_workspace_size(shape, R, C)
    assert need > 0 and L.lfbp_grad_psf_workspace_size(Shape(4, 5, 3, 3, 1), R, C) == 0
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, dH, None, need, None) == _abi.EINVAL
    assert L.lfbp_grad_psf_ws(None, g, shape, R, C, dH, 0x10000000, need, None) == _abi.EINVAL
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, w + 16, 0x10000000, need, None) == _abi.EALIAS
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, g + 16, 0x10000000, need, None) == _abi.EALIAS
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, dH + 2, 0x10000000, need, None) == _abi.EALIGN
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, dH, dH + 256, need, None) == _abi.EALIAS
    assert L.lfbp_grad_psf_ws(w, g, shape, R, C, dH, 0x10000000, need - 1, None) == _abi.EINVAL
    assert L.lfbp_grad_psf(w, g, Shape(15, 14, 3, 3, 3), R, C, dH, None) == _abi.ESHAPE
    assert L.lfbp_grad_psf(w, g, shape, R, C, g, None) == _abi.EALIAS


def test_colmajor_validation_before_launch():
    L = _abi.lib()
    assert L.lfbp_compute_Ht_colmajor(None, P2, GOOD, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_colmajor(P1, None, GOOD, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_colmajor(P1, P2, GOOD, 7, None) == _abi.EDTYPE
    assert L.lfbp_compute_Ht_colmajor(P1, P2, Shape(15, 14, 3, 3, 3), _abi.F32, None) == _abi.ESHAPE
    assert L.lfbp_compute_Ht_colmajor(P1 + 2, P2, GOOD, _abi.F32, None) == _abi.EALIGN
    assert L.lfbp_compute_Ht_colmajor(P1, P1 + 64, GOOD, _abi.F32, None) == _abi.EALIAS
    # cells of more than 2048 rows
    assert L.lfbp_compute_Ht_colmajor(P1, P2, Shape(3, 3, 2049, 1, 1), _abi.F16, None) == _abi.ESHAPE
    # nt * ny * nz * ns >= 2^31: at most one workgroup per position of every plane
    assert L.lfbp_compute_Ht_colmajor(P1, 1 << 44, Shape(4097, 3, 1, 1, 174763), _abi.F16, None) == _abi.ESHAPE


def test_operator_validation_before_launch():
    L = _abi.lib()
    shape, R, C = GOOD, 30, 30
    opb = L.lfbp_operator_size(shape, R, C)
    wsb = L.lfbp_operator_workspace_size(shape, R, C)
    assert opb > 0 and wsb > 0
    assert L.lfbp_operator_size(Shape(4, 5, 3, 3, 1), R, C) == 0
    assert L.lfbp_operator_workspace_size(shape, 0, C) == 0
    # the operator holds both packed PSFs: more than either unprepared call's records
    H, Ht, op, ws, g, f, n = 0x1000000, 0x2000000, 0x10000000, 0x20000000, 0x3000000, 0x4000000, 0x5000000
    assert L.lfbp_operator_prepare(None, Ht, shape, R, C, op, opb, None) == _abi.EINVAL
    assert L.lfbp_operator_prepare(H, Ht, shape, R, C, op, opb - 1, None) == _abi.EINVAL
    assert L.lfbp_operator_prepare(H, Ht, shape, R, C, op + 16, opb, None) == _abi.EINVAL
    assert L.lfbp_operator_prepare(H + 2, Ht, shape, R, C, op, opb, None) == _abi.EALIGN
    assert L.lfbp_operator_prepare(H, Ht, shape, R, C, H - 256, opb, None) == _abi.EALIAS
    assert L.lfbp_operator_prepare(H, Ht, Shape(15, 14, 3, 3, 3), R, C, op, opb, None) == _abi.ESHAPE
    # calls on the operator
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, f, ws, wsb - 1, None) == _abi.EINVAL
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, f, None, wsb, None) == _abi.EINVAL
    assert L.lfbp_forward_op(None, opb, shape, g, R, C, f, ws, wsb, None) == _abi.EINVAL
    assert L.lfbp_forward_op(op, opb, shape, None, R, C, f, ws, wsb, None) == _abi.EINVAL
    assert L.lfbp_forward_op(op, opb, shape, g + 2, R, C, f, ws, wsb, None) == _abi.EALIGN
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, g + 64, ws, wsb, None) == _abi.EALIAS     # f inside g
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, op + 64, ws, wsb, None) == _abi.EALIAS    # f inside op
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, f, op + 256, wsb, None) == _abi.EALIAS   # ws inside op
    assert L.lfbp_forward_op(op, opb, shape, g, R, C, f, g - 256, wsb, None) == _abi.EALIAS    # ws over g
    assert L.lfbp_backward_op(op, opb, shape, f, R, C, f + 64, ws, wsb, None) == _abi.EALIAS   # g over f
    assert L.lfbp_backward_op(op, opb, Shape(15, 15, 3, 3, 3), f, 0, C, g, ws, wsb, None) == _abi.EINVAL
    # Richardson-Lucy: g_out may be g, must not overlap anything else
    assert L.lfbp_rl_step_op(op, opb, shape, f, R, C, g, n, n + 64, ws, wsb, None) == _abi.EALIAS
    assert L.lfbp_rl_step_op(op, opb, shape, f, R, C, g, n, g + 64, ws, wsb, None) == _abi.EALIAS
    assert L.lfbp_rl_step_op(op, opb, shape, f, R, C, g, n, g, g - 256, wsb, None) == _abi.EALIAS
    assert L.lfbp_rl_norm_op(op, opb, shape, R, C, ws + 256, ws, wsb, None) == _abi.EALIAS
    assert L.lfbp_rl_norm_op(op, opb, shape, R, C, None, ws, wsb, None) == _abi.EINVAL


def test_noalloc_batch_limit_and_checks_before_any_hip_call():
    """lfbp_compute_Ht_batched_noalloc refuses a batch larger than its fixed
    scratch (ESCRATCH) and every bad table, all before touching a device."""
    L = _abi.lib()
    n = _abi.NOALLOC_MAX_PROBLEMS + 1
    nbytes = 15 * 15 * 3 * 3 * 3 * 4
    probs = (Problem * n)(*[Problem(P1, P2 + i * nbytes, GOOD) for i in range(n)])
    assert L.lfbp_compute_Ht_batched_noalloc(probs, n, _abi.F32, None) == _abi.ESCRATCH
    assert L.lfbp_compute_Ht_batched_noalloc(probs, 0, _abi.F32, None) == _abi.EINVAL
    assert L.lfbp_compute_Ht_batched_noalloc(None, 3, _abi.F32, None) == _abi.EINVAL
    bad = (Problem * 2)(Problem(P1, P2, GOOD), Problem(P1, P2, Shape(15, 14, 3, 3, 3)))
    assert L.lfbp_compute_Ht_batched_noalloc(bad, 2, _abi.F32, None) == _abi.ESHAPE
    alias = (Problem * 2)(Problem(P1, P2, GOOD), Problem(P1, P2 + 8, GOOD))
    assert L.lfbp_compute_Ht_batched_noalloc(alias, 2, _abi.F32, None) == _abi.EALIAS
    assert L.lfbp_compute_Ht_batched_noalloc(probs, 2, 9, None) == _abi.EDTYPE
