"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
entry point declared in include/ibm.h, the ctypes structures match the C layout
(compiled with gcc from the header), and invalid descriptors are rejected before
any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibm.h")
LIB = os.path.join(ROOT, "paper_2506_14328_amd", "libibm.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z_0-9]+)\s*\(", txt)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libibm.so not built")


@needs_lib
def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2506_14328_amd.ibm import EXPORTED
    assert sorted(EXPORTED) == names


def test_struct_layout_matches_c():
    from paper_2506_14328_amd.ibm import IbmGridDesc, IbmStats
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "ibm.h"
#define OFF(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("ibm_grid_desc size %zu\n", sizeof(ibm_grid_desc));
  printf("ibm_stats_t size %zu\n", sizeof(ibm_stats_t));
  OFF(ibm_grid_desc, nx); OFF(ibm_grid_desc, ibm); OFF(ibm_grid_desc, lx); OFF(ibm_grid_desc, q_target_or_pi);
  OFF(ibm_grid_desc, top); OFF(ibm_grid_desc, projection); OFF(ibm_grid_desc, pcg_max_iter);
  OFF(ibm_grid_desc, pcg_tol);
  OFF(ibm_stats_t, ke); OFF(ibm_stats_t, n_internal); OFF(ibm_stats_t, n_p_internal); OFF(ibm_stats_t, nan_flag);
  OFF(ibm_stats_t, pcg_iters);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe], text=True).split("\n")
    vals = {}
    for line in out:
        if line.strip():
            t, f, v = line.split()
            vals[(t, f)] = int(v)
    assert vals[("ibm_grid_desc", "size")] == ctypes.sizeof(IbmGridDesc)
    assert vals[("ibm_stats_t", "size")] == ctypes.sizeof(IbmStats)
    for (t, f), v in vals.items():
        if f == "size":
            continue
        cls = IbmGridDesc if t == "ibm_grid_desc" else IbmStats
        assert getattr(cls, f).offset == v, (t, f)


@needs_lib
@pytest.mark.parametrize("bad", [
    dict(nx=7), dict(nx=14), dict(nz=7), dict(ny=2), dict(dt=0.0), dict(nu=-1.0), dict(y_hi=-2.0),
    dict(forcing=3), dict(b_mode=9), dict(nx=2048), dict(top=2), dict(projection=2), dict(precision=2),
])
def test_invalid_descriptor_rejected(bad):
    from paper_2506_14328_amd.ibm import IBM_ERR_ARG, IbmGridDesc
    lib = ctypes.CDLL(LIB)
    d = dict(nx=8, ny=5, nz=4, forcing=0, b_mode=0, ibm=1, lx=1.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.01,
             dt=0.01, q_target_or_pi=1.0)
    d.update(bad)
    precision = d.pop("precision", 0)
    desc = IbmGridDesc(**d)
    h = ctypes.c_void_p()
    lib.ibm_create_grid.argtypes = [ctypes.POINTER(IbmGridDesc), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    rc = lib.ibm_create_grid(ctypes.byref(desc), 1, precision, None, ctypes.byref(h))
    assert rc == IBM_ERR_ARG
    assert not h.value


@needs_lib
def test_stream_kernels_validate_arguments():
    """ibm_stream_copy and ibm_stream_mix reject null, misaligned or overlapping arrays,
    counts outside 1..8 and sizes that are not multiples of 16 before any device work (the
    addresses below are never dereferenced)."""
    from paper_2506_14328_amd.ibm import IBM_ERR_ARG
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.ibm_stream_copy.argtypes = [vp, vp, ctypes.c_int64, vp]
    P = ctypes.POINTER(vp)
    lib.ibm_stream_mix.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int64, vp]
    A, B = 0x100000, 0x200000
    assert lib.ibm_stream_copy(None, vp(A), 64, None) == IBM_ERR_ARG
    assert lib.ibm_stream_copy(vp(B + 8), vp(A), 64, None) == IBM_ERR_ARG      # misaligned
    assert lib.ibm_stream_copy(vp(B), vp(A), 40, None) == IBM_ERR_ARG          # not 16k
    assert lib.ibm_stream_copy(vp(A + 32), vp(A), 64, None) == IBM_ERR_ARG     # overlap

    def arr(*xs):
        return (vp * len(xs))(*[vp(x) for x in xs])
    assert lib.ibm_stream_mix(None, 1, arr(A), 1, 64, None) == IBM_ERR_ARG
    assert lib.ibm_stream_mix(arr(B), 0, arr(A), 1, 64, None) == IBM_ERR_ARG
    assert lib.ibm_stream_mix(arr(*[B + 0x1000 * q for q in range(9)]), 9, arr(A), 1, 64, None) == IBM_ERR_ARG
    assert lib.ibm_stream_mix(arr(B), 1, arr(A), 1, 24, None) == IBM_ERR_ARG
    assert lib.ibm_stream_mix(arr(B + 4), 1, arr(A), 1, 64, None) == IBM_ERR_ARG
    assert lib.ibm_stream_mix(arr(B), 1, arr(B + 48), 1, 64, None) == IBM_ERR_ARG        # output on input
    assert lib.ibm_stream_mix(arr(B, B + 32), 2, arr(A), 1, 64, None) == IBM_ERR_ARG     # outputs overlap
    assert lib.ibm_last_error(None)


@needs_lib
def test_c_program_links_and_validates():
    """A C program built against include/ibm.h and linked with the library (no Python in
    between) names the kernels and gets IBM_ERR_ARG, with a message, for a descriptor the
    library rejects before any device work."""
    src = r'''
#include <stdio.h>
#include <string.h>
#include "ibm.h"
int main(void) {
  int n = ibm_num_kernels();
  if (n < 8 || strcmp(ibm_kernel_name(0), "momentum") != 0) return 1;
  ibm_grid_desc d;
  memset(&d, 0, sizeof d);
  d.nx = 7; d.ny = 5; d.nz = 4; d.lx = 1.0; d.lz = 1.0; d.y_lo = -1.0; d.y_hi = 1.0;
  d.nu = 0.01; d.dt = 0.01; d.ibm = 1;
  ibm_handle h = 0;
  int rc = ibm_create_grid(&d, 1, IBM_FP64, NULL, &h);
  if (rc != IBM_ERR_ARG || h != NULL) return 2;
  if (strlen(ibm_last_error(NULL)) == 0) return 3;
  printf("%d %s\n", n, ibm_last_error(NULL));
  return 0;
}
'''
    libdir = os.path.dirname(LIB)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe, "-L", libdir, "-libm",
                               "-Wl,-rpath," + libdir])
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "nx" in r.stdout


@needs_lib
def test_noalloc_binding_rejects_a_stretched_grid():
    """The allocation-free solve has no wall-normal table: its binding refuses a case with
    y_faces before touching any tensor."""
    import torch
    import ibm_inputs as I
    from paper_2506_14328_amd import solve_pressure_noalloc
    c = I.Case(nx=8, ny=9, nz=4, lx=1.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.01, dt=0.01,
               y_faces=I.tanh_faces(9, -1.0, 1.0, 1.2))
    with pytest.raises(ValueError):
        solve_pressure_noalloc(c, torch.zeros((8, 4, 8), dtype=torch.float64))
