"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes its workspace and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

import paper_1501_07293_amd as mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmag.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mm.LIB_PATH):
        from paper_1501_07293_amd import build
        build.build()
    return mm.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mm.EXPORTS)


def q(lib, nx, ny, nz, cell=5e-9, prec=0, pad=(0, 0, 0), threads=0, flags=0):
    g = mm.Grid(nx, ny, nz, cell)
    o = mm.Options(prec, pad[0], pad[1], pad[2], flags, threads, 0)
    b = ctypes.c_size_t()
    st = lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(o), ctypes.byref(b))
    return st, b.value


def test_workspace_query_sizes(lib):
    st, b32 = q(lib, 512, 512, 16)
    assert st == 0
    st, b64 = q(lib, 512, 512, 16, prec=1)
    assert st == 0 and b64 > b32
    # the working set of the 4.19M-cell film (FP32) stays far below one GPU's HBM
    assert b32 < 4 << 30
    st, b = q(lib, 1, 1, 1)
    assert st == 0 and b > 0


def test_autotune_workspace_covers_every_candidate(lib):
    st, plain = q(lib, 65, 33, 3)
    st2, tuned = q(lib, 65, 33, 3, flags=mm.MM_AUTOTUNE)
    st3, pow2 = q(lib, 65, 33, 3, pad=(256, 128, 8))
    assert st == st2 == st3 == 0
    assert tuned >= max(plain, pow2)


def test_batch_workspace_query(lib):
    grids = (mm.Grid * 3)(mm.Grid(32, 40, 1, 5e-9), mm.Grid(77, 33, 2, 5e-9), mm.Grid(1, 1, 1, 5e-9))
    o = mm.Options(0, 0, 0, 0, 0, 0, 0)
    b = ctypes.c_size_t()
    assert lib.mm_batch_workspace_query(3, grids, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value > 0
    bad = (mm.Grid * 2)(mm.Grid(32, 40, 1, 5e-9), mm.Grid(0, 33, 2, 5e-9))
    assert lib.mm_batch_workspace_query(2, bad, ctypes.byref(o), ctypes.byref(b)) == -1
    assert b"grid 1" in lib.mm_last_error()
    assert lib.mm_batch_workspace_query(0, grids, ctypes.byref(o), ctypes.byref(b)) == -1


def test_batch_autotune_workspace_covers_every_layout(lib):
    grids = (mm.Grid * 3)(mm.Grid(33, 47, 1, 5e-9), mm.Grid(77, 33, 2, 5e-9), mm.Grid(20, 20, 3, 5e-9))
    sizes = {}
    for name, flags in (("plain", 0), ("pow2", mm.MM_POW2_PAD),
                        ("pow2_generic", mm.MM_POW2_PAD | mm.MM_GENERIC_FFT), ("tuned", mm.MM_AUTOTUNE)):
        o = mm.Options(0, 0, 0, 0, flags, 0, 0)
        b = ctypes.c_size_t()
        assert lib.mm_batch_workspace_query(3, grids, ctypes.byref(o), ctypes.byref(b)) == 0
        sizes[name] = b.value
    assert sizes["tuned"] >= max(sizes["plain"], sizes["pow2"], sizes["pow2_generic"])
    assert sizes["pow2"] > sizes["plain"]
    info = mm.BatchInfo()
    assert lib.mm_batch_get_info(None, ctypes.byref(info)) == -1
    assert lib.mm_batch_get_grid_plan(None, 0, ctypes.byref(mm.PlanInfo())) == -1


@pytest.mark.parametrize("args", [(0, 4, 4), (4, -1, 4), (4, 4, 0)])
def test_workspace_query_rejects_bad_dims(lib, args):
    st, _ = q(lib, *args)
    assert st == -1
    assert b"dims" in lib.mm_last_error()


def test_workspace_query_rejects_bad_options(lib):
    assert q(lib, 8, 8, 1, cell=0.0)[0] == -1
    assert q(lib, 8, 8, 1, cell=float("nan"))[0] == -1
    assert q(lib, 8, 8, 1, prec=7)[0] == -1
    assert q(lib, 8, 8, 2, pad=(11, 0, 0))[0] == -1      # 11 is not 7-smooth
    assert q(lib, 8, 8, 2, pad=(14, 0, 0))[0] == -1      # below 2n-1 = 15
    assert q(lib, 8, 8, 2, pad=(15, 0, 0))[0] == 0       # 15 = 3*5 is allowed
    assert q(lib, 8, 8, 2, pad=(0, 0, 1))[0] == -1       # pz = 1 needs nz = 1
    assert q(lib, 8, 8, 2, threads=100)[0] == -1


def test_create_rejects_bad_material_without_gpu_work(lib):
    g = mm.Grid(8, 8, 1, 5e-9)
    o = mm.Options(0, 0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    for mat in (mm.Material(-1, 1e-11, 0, 0.5, 2.2e5), mm.Material(8e5, -1, 0, 0.5, 2.2e5),
                mm.Material(8e5, 1e-11, 0, -0.1, 2.2e5), mm.Material(8e5, 1e-11, 0, 0.5, 0.0),
                mm.Material(8e5, 1e-11, float("inf"), 0.5, 2.2e5)):
        st = lib.mm_create(ctypes.byref(g), ctypes.byref(mat), ctypes.byref(o), None, 0, None,
                           ctypes.byref(h))
        assert st == -1
        assert not h.value
    # undersized caller workspace
    mat = mm.Material(8e5, 1.3e-11, 0, 0.5, 2.2e5)
    st = lib.mm_create(ctypes.byref(g), ctypes.byref(mat), ctypes.byref(o), 256, 16, None,
                       ctypes.byref(h))
    assert st == -1 and b"workspace" in lib.mm_last_error()


def test_null_handles_are_rejected(lib):
    assert lib.mm_destroy(None) == 0
    assert lib.mm_step(None, 1, 1e-13) == -1
    assert lib.mm_set_m(None, None, 0) == -1
    assert lib.mm_get_energy(None, None) == -1
    assert lib.mm_demag_tensor(0, 1, 1, None, None) == -1
    assert lib.mm_status_string(-6) == b"MM_ENONFINITE"
    assert lib.mm_kernel_name(2) == b"k_kspace"


def test_product_has_no_cpu_fallback():
    # The package never imports the oracle.
    import inspect
    src = inspect.getsource(mm)
    assert "oracle" not in src
    pkg = os.path.dirname(mm.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                assert "import oracle" not in open(os.path.join(root, f)).read()


def test_batch_create_rejects_bad_arguments_without_gpu_work(lib):
    grids = (mm.Grid * 2)(mm.Grid(32, 40, 1, 5e-9), mm.Grid(40, 33, 2, 5e-9))
    o = mm.Options(0, 0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    bad_mat = mm.Material(8e5, 1.3e-11, 0, -1.0, 2.2e5)
    assert lib.mm_batch_create(2, grids, ctypes.byref(bad_mat), None, ctypes.byref(o), None, 0, None,
                               ctypes.byref(h)) == -1
    mat = mm.Material(8e5, 1.3e-11, 500.0, 0.5, 2.2e5)
    hext = (ctypes.c_double * 6)(0, 0, 0, float("nan"), 0, 0)
    assert lib.mm_batch_create(2, grids, ctypes.byref(mat), hext, ctypes.byref(o), None, 0, None,
                               ctypes.byref(h)) == -1
    assert lib.mm_batch_create(2, grids, ctypes.byref(mat), None, ctypes.byref(o), 256, 16, None,
                               ctypes.byref(h)) == -1
    assert b"workspace" in lib.mm_last_error()
    assert not h.value
    assert lib.mm_batch_destroy(None) == 0
    assert lib.mm_batch_step(None, 1, 1e-13) == -1


def test_periodic_options_validated_without_gpu_work(lib):
    b = ctypes.c_size_t()
    g = mm.Grid(64, 48, 4, 5e-9)
    per = mm.MM_PERIODIC_X | mm.MM_PERIODIC_Y
    ok = mm.Options(0, 0, 0, 0, per, 0, 0, 2)
    assert lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(ok), ctypes.byref(b)) == 0
    padded = mm.Options(0, 0, 0, 0, 0, 0, 0, 0)
    b2 = ctypes.c_size_t()
    assert lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(padded), ctypes.byref(b2)) == 0
    assert b.value < b2.value                          # no zero padding along x and y
    bad_size = mm.Options(0, 128, 0, 0, mm.MM_PERIODIC_X, 0, 0, 0)
    assert lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(bad_size), ctypes.byref(b)) == -1
    assert lib.mm_workspace_query(ctypes.byref(mm.Grid(22, 8, 1, 5e-9)),
                                  ctypes.byref(mm.Options(0, 0, 0, 0, mm.MM_PERIODIC_X, 0, 0, 0)),
                                  ctypes.byref(b)) == -5          # 22 = 2 x 11 is not 7-smooth
    assert lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(mm.Options(0, 0, 0, 0, per, 0, 0, 65)),
                                  ctypes.byref(b)) == -1
    grids = (mm.Grid * 2)(mm.Grid(32, 40, 1, 5e-9), mm.Grid(40, 33, 2, 5e-9))
    assert lib.mm_batch_workspace_query(2, grids, ctypes.byref(mm.Options(0, 0, 0, 0, per, 0, 0, 0)),
                                        ctypes.byref(b)) == -5
    for dims in ((1, 16, 4), (8, 1, 3)):          # one-cell periods along x or y
        assert lib.mm_workspace_query(ctypes.byref(mm.Grid(*dims, 5e-9)), ctypes.byref(ok),
                                      ctypes.byref(b)) == -5
    assert lib.mm_workspace_query(ctypes.byref(mm.Grid(6, 5, 1, 5e-9)),
                                  ctypes.byref(mm.Options(0, 0, 0, 0, mm.MM_PERIODIC_Z, 0, 0, 2)),
                                  ctypes.byref(b)) == 0


def test_profile_entry_points_reject_bad_arguments(lib):
    assert lib.mm_profile_begin(None, 2) == -1
    assert lib.mm_profile_sample(None, 4) == -1
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.mm_profile_end(None, ctypes.byref(ms), ctypes.byref(n)) == -1


def test_adjoint_and_euler_entry_points_reject_null(lib):
    assert lib.mm_step_euler(None, 1, 1e-13) == -1
    assert lib.mm_rollout(None, 10, 1e-13, 5, None) == -1
    b = ctypes.c_size_t()
    assert lib.mm_adjoint_workspace_query(None, 5, ctypes.byref(b)) == -1
    assert lib.mm_backward(None, 10, 1e-13, 5, None, None, None, None, None, 0) == -1
    assert lib.mm_backward_noalloc(None, 10, 1e-13, 5, None, None, None, None) == -1


def test_noalloc_scratch_size_matches_the_header():
    text = open(HEADER).read()
    shift = re.search(r"#define MM_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert shift, "MM_NOALLOC_SCRATCH_BYTES not found"
    assert int(shift.group(1)) << int(shift.group(2)) == mm.MM_NOALLOC_SCRATCH_BYTES


def test_x_lines_option_validated(lib):
    g = mm.Grid(64, 64, 4, 5e-9)
    b = ctypes.c_size_t()
    for xl, want in ((0, 0), (4, 0), (8, 0), (16, 0), (6, -1), (32, -1)):
        o = mm.Options(0, 0, 0, 0, 0, 0, xl)
        assert lib.mm_workspace_query(ctypes.byref(g), ctypes.byref(o), ctypes.byref(b)) == want


def test_schedule_and_newell_entry_points_reject_bad_arguments(lib):
    seg = (mm.Segment * 1)()
    seg[0].steps = 5
    rows = ctypes.c_int64(7)
    assert lib.mm_run_schedule(None, seg, 1, mm.MM_RK4, 1e-14, 1, None, 0, ctypes.byref(rows)) == -1
    assert rows.value == 0
    assert lib.mm_demag_tensor_newell(0, 1, 1, None, None) == -1
    assert lib.mm_demag_tensor_newell(2, 2, 2, None, None) == -1
    assert b"dims" in lib.mm_last_error()


def test_batch_per_grid_materials_validated_without_gpu_work(lib):
    grids = (mm.Grid * 2)(mm.Grid(32, 40, 1, 5e-9), mm.Grid(40, 33, 2, 5e-9))
    o = mm.Options(0, 0, 0, 0, mm.MM_PER_GRID_MATERIAL, 0, 0)
    mats = (mm.Material * 2)(mm.Material(8e5, 1.3e-11, 0, 0.5, 2.2e5), mm.Material(8e5, 1.3e-11, 0, -0.5, 2.2e5))
    h = ctypes.c_void_p()
    assert lib.mm_batch_create(2, grids, mats, None, ctypes.byref(o), None, 0, None, ctypes.byref(h)) == -1
    assert b"grid 1" in lib.mm_last_error()
    assert lib.mm_batch_create(2, grids, None, None, ctypes.byref(o), None, 0, None, ctypes.byref(h)) == -1



def test_binding_constants_match_the_header():
    # every MM_ flag and enum value the header defines, the binding defines alike;
    # the option flags are distinct single bits
    text = open(HEADER).read()
    flags = {k: int(v, 16) for k, v in re.findall(r"#define (MM_[A-Z0-9_]+) (0x[0-9a-fA-F]+)u", text)}
    assert len(flags) >= 12
    for k, v in flags.items():
        assert getattr(mm, k) == v, k
        assert v & (v - 1) == 0, k
    assert len(set(flags.values())) == len(flags)
    enums = dict(re.findall(r"\b(MM_F32|MM_F64|MM_RK4|MM_EULER)\s*=\s*(\d+)", text))
    assert {k: getattr(mm, k) for k in enums} == {k: int(v) for k, v in enums.items()}


def test_option_and_plan_structs_match_the_header():
    # the ctypes mirrors list the C structs' fields in order, with the same widths
    text = open(HEADER).read()

    def fields(name):
        end = text.index("} " + name + ";")
        body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            typ, names = decl.split(None, 1)
            for n in names.split(","):
                n = n.strip()
                m = re.match(r"(\w+)(?:\[(\d+)\])?", n)
                out.append((m.group(1), typ, int(m.group(2) or 1)))
        return out

    width = {"int32_t": 4, "uint32_t": 4, "int64_t": 8, "double": 8, "size_t": 8}
    for cname, py, same_names in (("mm_options", mm.Options, True), ("mm_plan_info", mm.PlanInfo, True),
                                  ("mm_grid", mm.Grid, True), ("mm_material", mm.Material, True),
                                  ("mm_segment", mm.Segment, True), ("mm_batch_info", mm.BatchInfo, False)):
        c = fields(cname)
        assert len(c) == len(py._fields_), cname
        if same_names:
            assert [n for n, _, _ in c] == [n for n, _ in py._fields_], cname
        for (n, typ, count), (_, ct) in zip(c, py._fields_):
            assert ctypes.sizeof(ct) == width[typ] * count, (cname, n)
