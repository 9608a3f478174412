"""The C ABI library: symbols and host-side argument checks (no GPU work:
every call below is rejected before anything is enqueued)."""
import ctypes as C
import os
import re

import pytest

import otm_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "otm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(otm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2206_08772_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    names = _declared()
    assert "otm_step" in names and "otm_build_neighbors" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(L.exported_symbols())


def test_status_strings_and_workspace_size(L):
    lib = L.lib()
    assert lib.otm_status_string(L.OTM_ERR_CAPACITY).startswith(b"OTM_ERR_CAPACITY")
    a = lib.otm_workspace_bytes(1000, 4000, 100000)
    b = lib.otm_workspace_bytes(1000, 4000, 200000)
    assert a > 0 and a % 256 == 0 and b - a >= 8 * 100000 - 512
    assert lib.otm_workspace_bytes(-1, 0, 0) == 0


def _fake_state(L, prec=0):
    s = L.State()
    s.n_nodes, s.n_mp, s.pair_capacity, s.precision = 10, 20, 100, prec
    for name, _ in L.State._fields_[5:]:
        setattr(s, name, 1 << 20)      # aligned non-null stand-ins, never dereferenced
    return s


def _params(L, **over):
    from paper_2206_08772_amd.sim import make_params
    w = W.elastic_cube(n=3)
    p = W.params_from_workload(w, **over)
    return make_params(p)


@pytest.mark.parametrize("bad", [
    dict(cell_size=0.5),            # cell edge below the search radius
    dict(model=7),
    dict(lme_tol=0.0),
    dict(nu=0.5),
])
def test_bad_params_are_rejected(L, bad):
    lib = L.lib()
    st = _fake_state(L)
    p = _params(L, **bad)
    code = lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None)
    assert code == L.OTM_ERR_ARG


def test_bad_state_and_workspace_are_rejected(L):
    lib = L.lib()
    p = _params(L)
    st = _fake_state(L)
    st.x = 0
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    st = _fake_state(L)
    st.N = (1 << 20) + 4           # misaligned double array
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    st = _fake_state(L)
    st.precision = 5
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    st = _fake_state(L)
    # workspace too small
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 64,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    # unknown scatter mode, non-positive time step
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 9, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    assert lib.otm_step(C.byref(st), C.byref(p), 0.0, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG
    # pair ids are int32
    st.pair_capacity = 1 << 31
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), 1 << 40,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG


def test_search_and_lme_argument_checks(L):
    lib = L.lib()
    n = C.c_int64(0)
    fake = C.c_void_p(1 << 20)
    # cell edge smaller than the radius
    assert lib.otm_build_neighbors(10, fake, 10, fake, 1.0, 0.5, 100, fake, fake, C.byref(n),
                                   fake, 1 << 30, None) == L.OTM_ERR_ARG
    # negative sizes, missing count pointer
    assert lib.otm_build_neighbors(-1, fake, 10, fake, 1.0, 1.0, 100, fake, fake, C.byref(n),
                                   fake, 1 << 30, None) == L.OTM_ERR_ARG
    assert lib.otm_build_neighbors(10, fake, 10, fake, 1.0, 1.0, 100, fake, fake, None,
                                   fake, 1 << 30, None) == L.OTM_ERR_ARG
    # LME: bad precision, non-positive beta or tolerance
    assert lib.otm_lme_shape(10, fake, 10, fake, fake, fake, 100, 4.0, 1e-13, 50, fake, fake,
                             fake, 3, None, None) == L.OTM_ERR_ARG
    assert lib.otm_lme_shape(10, fake, 10, fake, fake, fake, 100, -4.0, 1e-13, 50, fake, fake,
                             fake, 0, None, None) == L.OTM_ERR_ARG
    assert lib.otm_lme_shape(10, fake, 10, fake, fake, fake, 100, 4.0, 0.0, 50, fake, fake,
                             fake, 0, None, None) == L.OTM_ERR_ARG


def test_kernel_resource_parser():
    """The build refuses kernels that spill; the parser reads the compiler's
    kernel-resource-usage remarks (text in the form hipcc prints)."""
    from paper_2206_08772_amd.build import kernel_resources
    txt = "\n".join([
        "a.hip:1:1: remark: Function Name: k_one [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 120 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: k_two [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     AGPRs: 58 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     VGPRs Spill: 4 [-Rpass-analysis=kernel-resource-usage]",
    ])
    r = kernel_resources(txt)
    assert r["k_one"] == {"VGPRs": 120, "AGPRs": 0, "ScratchSize": 0, "VGPRs Spill": 0}
    assert r["k_two"] == {"VGPRs": 256, "AGPRs": 58, "ScratchSize": 16, "VGPRs Spill": 4}


def test_step_into_rejects_missing_misaligned_or_aliased_lists(L):
    """otm_step_into checks the target lists before anything is enqueued."""
    lib = L.lib()
    p = _params(L)
    st = _fake_state(L)
    ws, diag = C.c_void_p(1 << 20), C.c_void_p(1 << 20)

    def call(nxt):
        return lib.otm_step_into(C.byref(st), nxt, C.byref(p), 1e-3, 1, 0, ws, 1 << 30, diag,
                                 None)

    assert call(None) == L.OTM_ERR_ARG
    nxt = L.Lists()
    nxt.nbr_offsets, nxt.nbr_idx, nxt.N, nxt.dN = 2 << 20, 2 << 20, 2 << 20, (2 << 20) + 4
    assert call(C.byref(nxt)) == L.OTM_ERR_ARG          # misaligned float64 dN
    nxt.dN = 2 << 20
    nxt.N = st.N                                        # overlaps the state's N
    before = (st.nbr_offsets, st.nbr_idx, st.N, st.dN)
    assert call(C.byref(nxt)) == L.OTM_ERR_ARG
    assert (st.nbr_offsets, st.nbr_idx, st.N, st.dN) == before
    nxt.N, nxt.nbr_offsets = 2 << 20, 0                 # missing offsets
    assert call(C.byref(nxt)) == L.OTM_ERR_ARG


@pytest.mark.parametrize("bad", [
    dict(fracture=True, model=W.MODEL_J2_LINEAR),     # fracture needs the JC model
    dict(tool_r=0.0),
    dict(tool_clearance=1.6),
    dict(tool_mu=-0.1),
    dict(tool_cN=0.0),
])
def test_bad_cutting_params_are_rejected(L, bad):
    from paper_2206_08772_amd.sim import make_params
    lib = L.lib()
    w = W.config_by_name("small_cut")
    p = make_params(W.params_from_workload(w, **bad))
    st = _fake_state(L)
    assert lib.otm_step(C.byref(st), C.byref(p), 1e-10, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                        C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG


def test_cutting_needs_its_state_arrays(L):
    from paper_2206_08772_amd.sim import make_params
    lib = L.lib()
    w = W.config_by_name("small_cut")
    p = make_params(W.params_from_workload(w))
    for missing in ("failed", "tool_gt", "clock"):
        st = _fake_state(L)
        setattr(st, missing, 0)
        assert lib.otm_step(C.byref(st), C.byref(p), 1e-10, 1, 0, C.c_void_p(1 << 20), 1 << 30,
                            C.c_void_p(1 << 20), None) == L.OTM_ERR_ARG, missing
        assert lib.otm_init(C.byref(st), C.byref(p), 1e-10, C.c_void_p(1 << 20), 0,
                            C.c_void_p(1 << 20), 1 << 30, C.c_void_p(1 << 20),
                            None) == L.OTM_ERR_ARG, missing


def test_header_compiles_as_c_and_links(L, tmp_path):
    """include/otm.h is a C header: a C program that includes it, fills the
    structs and calls two host-only entry points compiles, links against
    libotm.so and runs (no device work)."""
    import shutil
    import subprocess
    from paper_2206_08772_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text("""
#include <stdio.h>
#include <string.h>
#include "otm.h"
int main(void) {
  otm_params p; otm_state st; otm_lists l; otm_tape t; otm_state_bar b; otm_diag d;
  memset(&p, 0, sizeof p); memset(&st, 0, sizeof st); memset(&l, 0, sizeof l);
  memset(&t, 0, sizeof t); memset(&b, 0, sizeof b); memset(&d, 0, sizeof d);
  size_t ws = otm_workspace_bytes(1000, 4000, 100000);
  const char* s = otm_status_string(OTM_ERR_CAPACITY);
  printf("%zu %zu %zu %zu %zu %zu %zu %s\\n", ws, sizeof(otm_params), sizeof(otm_state),
         sizeof(otm_lists), sizeof(otm_tape), sizeof(otm_state_bar), sizeof(otm_diag), s);
  return ws > 0 && s != NULL ? 0 : 1;
}
""")
    exe = tmp_path / "abi"
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = [gcc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", str(src), "-o", str(exe), "-L", libdir, "-lotm",
           f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    *sizes, status = r.stdout.split(maxsplit=7)
    ws, sizes = int(sizes[0]), [int(v) for v in sizes[1:]]
    assert ws == L.lib().otm_workspace_bytes(1000, 4000, 100000)
    assert status.startswith("OTM_ERR_CAPACITY")
    # the ctypes mirrors have the C sizes
    assert sizes == [C.sizeof(t) for t in (L.Params, L.State, L.Lists, L.Tape, L.StateBar,
                                            L.Diag)]


def test_erode_argument_checks(L):
    """otm_erode needs the fracture model, no stabilisation term, a place for
    the count and a known assembly; it rejects before enqueuing anything and
    leaves the state as it was."""
    from paper_2206_08772_amd.sim import make_params
    lib = L.lib()
    w = W.config_by_name("small_cut")
    ws, diag = C.c_void_p(1 << 20), C.c_void_p(1 << 20)
    n = C.c_int64(-1)

    def call(p, st, out=C.byref(n), mode=0):
        return lib.otm_erode(C.byref(st), C.byref(p), mode, ws, 1 << 30, diag, out, None, None)

    st = _fake_state(L)
    ok = make_params(W.params_from_workload(w))
    assert call(make_params(W.params_from_workload(w, fracture=False)), st) == L.OTM_ERR_ARG
    assert call(make_params(W.params_from_workload(w, eps_stab=1.0)), st) == L.OTM_ERR_ARG
    assert call(ok, st, out=None) == L.OTM_ERR_ARG
    assert call(ok, st, mode=7) == L.OTM_ERR_ARG
    assert lib.otm_erode(C.byref(st), C.byref(ok), 0, ws, 1 << 30, C.c_void_p(0), C.byref(n),
                         None, None) == L.OTM_ERR_ARG
    # node management: a negative insertion distance, an unknown flag, a
    # negative node capacity
    assert call(make_params(W.params_from_workload(w, insert_dist=-1.0)), st) == L.OTM_ERR_ARG
    bad = make_params(W.params_from_workload(w))
    bad.delete_orphans = 2
    assert call(bad, st) == L.OTM_ERR_ARG
    st.node_capacity = -5
    assert call(ok, st) == L.OTM_ERR_ARG
    st.node_capacity = 0
    st.failed = 0
    assert call(ok, st) == L.OTM_ERR_ARG
    assert n.value == -1 and st.n_mp == 20 and st.n_nodes == 10


def test_noalloc_step_rejects_states_larger_than_its_scratch(L):
    """otm_step_noalloc refuses, before any device work, a state whose
    workspace would exceed the static scratch."""
    lib = L.lib()
    p = _params(L)
    st = _fake_state(L)
    st.n_nodes, st.n_mp, st.pair_capacity = 200_000, 1_000_000, 30_000_000
    assert lib.otm_workspace_bytes(st.n_nodes, st.n_mp, st.pair_capacity) > \
        L.OTM_STATIC_SCRATCH_BYTES
    code = lib.otm_step_noalloc(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20), None)
    assert code == L.OTM_ERR_SCRATCH
    assert lib.otm_status_string(code).startswith(b"OTM_ERR_SCRATCH")
    st.x = 0                                   # argument errors come first
    assert lib.otm_step_noalloc(C.byref(st), C.byref(p), 1e-3, 1, 0, C.c_void_p(1 << 20),
                                None) == L.OTM_ERR_ARG
