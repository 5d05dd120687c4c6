"""The C ABI: the library loads without a GPU, exports every entry point that
include/*.h declares, and the ctypes structures match the C layout."""
import glob
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrcm.h")


def _declared_functions():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mrcm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_three_named_entry_points():
    names = _declared_functions()
    for n in ("mrcm_build_mbfs", "mrcm_assemble_interface", "mrcm_reconstruct"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_08513_amd import _lib
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == _declared_functions()


def test_library_exports_nothing_but_the_declared_abi():
    """The dynamic symbol table holds the declared entry points and no
    internal symbol (launchers, kernel stubs, host helpers)."""
    import shutil
    import subprocess
    from paper_2103_08513_amd import _lib
    nm = shutil.which("nm") or shutil.which("llvm-nm")
    if nm is None:
        pytest.skip("no nm on this host")
    out = subprocess.run([nm, "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    names = sorted(ln.split()[-1] for ln in out.splitlines() if ln.strip())
    assert names == _declared_functions()


def test_status_strings_without_gpu():
    from paper_2103_08513_amd import _lib
    lib = _lib.load()
    assert lib.mrcm_status_string(0) == b"ok"
    assert lib.mrcm_status_string(-7) == b"unsupported by this build"


def test_host_validation_rejects_bad_arguments_before_any_gpu_work():
    """Argument errors are caught on the host: no device is touched."""
    import numpy as np
    from paper_2103_08513_amd import _lib
    from paper_2103_08513_amd._lib import CIfaceSpace, COptions, CPartition, CProblem
    lib = _lib.load()
    pb = CProblem()
    pb.nx, pb.ny, pb.nz = 4, 4, 4
    pb.hx = pb.hy = pb.hz = 1.0
    pb.kx = pb.ky = pb.kz = pb.q = 8  # never dereferenced: validation fails first
    pb.pin_cell = -1                  # no pin and no Dirichlet wall -> EINVAL
    part = CPartition()
    part.ndx = part.ndy = part.ndz = 1
    ifs = CIfaceSpace()
    opt = COptions()
    opt.alpha = 1.0
    out = ctypes.c_void_p()
    code = lib.mrcm_build_mbfs(ctypes.byref(pb), ctypes.byref(part), ctypes.byref(ifs),
                               ctypes.byref(opt), None, ctypes.byref(out))
    assert code == -1
    assert b"pin" in lib.mrcm_last_error()
    pb.pin_cell = 0
    opt.alpha = -1.0
    code = lib.mrcm_build_mbfs(ctypes.byref(pb), ctypes.byref(part), ctypes.byref(ifs),
                               ctypes.byref(opt), None, ctypes.byref(out))
    assert code == -1 and b"alpha" in lib.mrcm_last_error()
    opt.alpha = 1.0
    cuts = np.array([0, 3, 3, 4], dtype=np.int32)
    part.ndx = 3
    part.cut_x = cuts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    code = lib.mrcm_build_mbfs(ctypes.byref(pb), ctypes.byref(part), ctypes.byref(ifs),
                               ctypes.byref(opt), None, ctypes.byref(out))
    assert code == -1 and b"cuts" in lib.mrcm_last_error()


def test_ctypes_layout_matches_c(tmp_path):
    """sizeof/offsetof of the ABI structs, from the C compiler, equal ctypes'."""
    from paper_2103_08513_amd._lib import CIfaceInfo, CInfo, CIfaceSpace, COptions, CPartition, CProblem, CSubInfo
    src = tmp_path / "layout.c"
    src.write_text(f'''
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu\\n", sizeof(mrcm_problem), offsetof(mrcm_problem, kx), offsetof(mrcm_problem, wall_type), offsetof(mrcm_problem, pin_cell));
  printf("%zu %zu\\n", sizeof(mrcm_partition), offsetof(mrcm_partition, cut_x));
  printf("%zu %zu\\n", sizeof(mrcm_iface_space), offsetof(mrcm_iface_space, split));
  printf("%zu %zu %zu %zu\\n", sizeof(mrcm_options), offsetof(mrcm_options, ir_tol), offsetof(mrcm_options, ir_max_iter), offsetof(mrcm_options, fp64_refine));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(mrcm_options, pcg_max_iter), offsetof(mrcm_options, pcg_x0), offsetof(mrcm_options, pcg_x0_scale), offsetof(mrcm_options, solve_tiles), offsetof(mrcm_options, solve_group));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(mrcm_info), offsetof(mrcm_info, ir_residual), offsetof(mrcm_info, device_bytes), offsetof(mrcm_info, pcg_fallback), offsetof(mrcm_info, pcg_iters));
  printf("%zu %zu %zu\\n", sizeof(mrcm_subdomain_info), offsetof(mrcm_subdomain_info, pin_local), offsetof(mrcm_subdomain_info, solve_group));
  printf("%zu %zu %zu %zu\\n", offsetof(mrcm_options, beta_mode), offsetof(mrcm_options, keep), offsetof(mrcm_options, iface_panel), offsetof(mrcm_options, launch_mode));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(mrcm_interface_info), offsetof(mrcm_interface_info, front_bytes), offsetof(mrcm_interface_info, factor_flops), offsetof(mrcm_interface_info, device_bytes), offsetof(mrcm_interface_info, rel_residual));
  return 0;
}}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    got = [list(map(int, ln.split())) for ln in subprocess.check_output([str(exe)]).decode().splitlines()]
    want = [
        [ctypes.sizeof(CProblem), CProblem.kx.offset, CProblem.wall_type.offset, CProblem.pin_cell.offset],
        [ctypes.sizeof(CPartition), CPartition.cut_x.offset],
        [ctypes.sizeof(CIfaceSpace), CIfaceSpace.split.offset],
        [ctypes.sizeof(COptions), COptions.ir_tol.offset, COptions.ir_max_iter.offset,
         COptions.fp64_refine.offset],
        [COptions.pcg_max_iter.offset, COptions.pcg_x0.offset, COptions.pcg_x0_scale.offset,
         COptions.solve_tiles.offset, COptions.solve_group.offset],
        [ctypes.sizeof(CInfo), CInfo.ir_residual.offset, CInfo.device_bytes.offset, CInfo.pcg_fallback.offset,
         CInfo.pcg_iters.offset],
        [ctypes.sizeof(CSubInfo), CSubInfo.pin_local.offset, CSubInfo.solve_group.offset],
        [COptions.beta_mode.offset, COptions.keep.offset, COptions.iface_panel.offset, COptions.launch_mode.offset],
        [ctypes.sizeof(CIfaceInfo), CIfaceInfo.front_bytes.offset, CIfaceInfo.factor_flops.offset,
         CIfaceInfo.device_bytes.offset, CIfaceInfo.rel_residual.offset],
    ]
    assert got == want


def test_host_validation_of_the_forms_and_tunables():
    """Option, size and network-argument errors are caught on the host."""
    from paper_2103_08513_amd import _lib
    from paper_2103_08513_amd._lib import CIfaceSpace, COptions, CPartition, CProblem
    lib = _lib.load()
    pb = CProblem()
    pb.nx, pb.ny, pb.nz = 2, 40, 30   # one 2400-cell block, bandwidth 60
    pb.hx = pb.hy = pb.hz = 1.0
    pb.kx = pb.ky = pb.kz = pb.q = 8  # never dereferenced
    pb.pin_cell = 0
    part = CPartition()
    part.ndx = part.ndy = part.ndz = 1
    ifs = CIfaceSpace()
    opt = COptions()
    opt.alpha = 1.0
    out = ctypes.c_void_p()

    def build():
        return lib.mrcm_build_mbfs(ctypes.byref(pb), ctypes.byref(part), ctypes.byref(ifs),
                                   ctypes.byref(opt), None, ctypes.byref(out))

    opt.solve_tiles = 4
    assert build() == -1 and b"solve_tiles" in lib.mrcm_last_error()
    opt.solve_tiles = 0
    opt.solve_group = -2
    assert build() == -1 and b"solve_group" in lib.mrcm_last_error()
    opt.solve_group = 0
    opt.iface_panel = 5
    assert build() == -1 and b"iface_panel" in lib.mrcm_last_error()
    opt.iface_panel = -1
    assert build() == -1 and b"iface_panel" in lib.mrcm_last_error()
    opt.iface_panel = 0
    opt.launch_mode = 2
    assert build() == -1 and b"launch_mode" in lib.mrcm_last_error()
    opt.launch_mode = 0
    opt.beta_mode = 2
    assert build() == -1 and b"beta_mode" in lib.mrcm_last_error()
    opt.beta_mode = 1
    opt.keep = 4
    assert build() == -1 and b"keep" in lib.mrcm_last_error()
    opt.keep = 2 | 1
    opt.precision = 2
    opt.keep = 1                  # re-solve without MBFs needs factors the CG form does not keep
    assert build() == -1 and b"conjugate-gradient form keeps no factors" in lib.mrcm_last_error()
    opt.keep = 0
    opt.beta_mode = 0
    opt.precision = 3
    assert build() == -1 and b"precision" in lib.mrcm_last_error()
    opt.precision = 2             # conjugate gradients: at most 2048 cells per block
    assert build() == -7 and b"conjugate-gradient" in lib.mrcm_last_error()
    # the local bandwidth (product of the two shortest extents) above each
    # form's largest: 112 in FP64, 176 in FP32
    opt.precision = 0
    pb.ny, pb.nz = 57, 60         # bandwidth 114
    assert build() == -7 and b"local bandwidth 114 exceeds 112" in lib.mrcm_last_error()
    opt.precision = 1
    pb.ny, pb.nz = 89, 100        # bandwidth 178
    assert build() == -7 and b"local bandwidth 178 exceeds 176" in lib.mrcm_last_error()
    pb.ny, pb.nz = 40, 30
    # network kernels: channel limit and sizes
    nul = ctypes.c_void_p(8)
    assert lib.mrcm_conv3d_max_channels() == 16
    assert lib.mrcm_conv3d_forward(nul, nul, None, nul, None, 1, 17, 1, 2, 2, 2, 1, 0, None) == -1
    assert lib.mrcm_conv3d_forward(nul, nul, None, nul, None, 1, 2, 1, 0, 2, 2, 1, 0, None) == -1
    assert lib.mrcm_conv3d_forward(nul, nul, None, nul, None, 1, 2, 1, 2, 2, 2, 0, 0, None) == -1
    assert lib.mrcm_adam_step(nul, nul, nul, nul, 4, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    # graph capture and autotuning need handles and arguments
    g = ctypes.c_void_p()
    assert lib.mrcm_graph_capture(None, None, None, None, None, None, 0, None, None, None, None,
                                  ctypes.byref(g)) == -1
    assert lib.mrcm_graph_launch(None, None) == -1
    assert lib.mrcm_autotune(None, None, None, None, None, None, None, None) == -1
    # interface solve arguments
    assert lib.mrcm_solve_interface(None, 0, 0.0, 0, None, None, None, None) == -1
    assert lib.mrcm_interface_query(None, None) == -1


def test_binding_refuses_wall_data_of_the_wrong_length():
    """Checked in the constructor, before any device memory is touched."""
    import numpy as np
    from mrcm_inputs import small_case
    import paper_2103_08513_amd as lib
    case = small_case((8, 6, 4), (2, 2, 2), seed=1, pin=-1)
    pb = case.problem
    pb.wall_type = [1, 0, 0, 0, 0, 0]
    pb.wall_value = [np.zeros(6 * 4 - 1), None, None, None, None, None]
    with pytest.raises(ValueError):
        lib.MRCM(pb, case.partition, case.iface)
