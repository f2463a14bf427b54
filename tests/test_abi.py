"""The C-ABI library loads, exports every symbol include/qed.h declares, and validates its
arguments on the host (no GPU needed: no compute call is made)."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qed.h")


@pytest.fixture(scope="module")
def Q():
    from paper_1412_6426_amd import build, qed
    if not os.path.exists(qed.LIB_PATH):
        build.build()
    qed.lib()
    return qed


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qed_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for must in ("qed_build_tables", "qed_step", "qed_append_stats"):
        assert must in names


def test_every_declared_symbol_is_exported(Q):
    lib = C.CDLL(Q.LIB_PATH)
    names = declared_functions()
    assert set(names) == set(Q.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_ctypes_layout_matches_header(Q, tmp_path):
    """Compile a probe against include/qed.h with gcc and compare every struct's size and
    every field's offset with the ctypes mirror."""
    structs = [Q.qed_soa, Q.qed_instance, Q.qed_stores, Q.qed_field, Q.qed_params, Q.qed_stats,
               Q.qed_thin_record, Q.qed_thin_cells_record, Q.qed_thin_children_record,
               Q.qed_schwinger_record]
    lines = ['#include "qed.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void){"]
    expect = []
    for S in structs:
        lines.append(f'printf("%zu\\n", sizeof({S.__name__}));')
        expect.append(C.sizeof(S))
        for name, _ in S._fields_:
            lines.append(f'printf("%zu\\n", offsetof({S.__name__}, {name}));')
            expect.append(getattr(S, name).offset)
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == expect
    assert Q.qed_table_bytes() == 221696


def test_host_side_queries(Q):
    assert Q.qed_version() >= 100
    assert Q.qed_work_bytes(0, 10) == 0
    assert Q.qed_work_bytes(1, -1) == 0
    assert Q.qed_work_bytes(1, 10, -1) == 0
    w1, w64 = Q.qed_work_bytes(1, 1000), Q.qed_work_bytes(64, 1000)
    assert 64 <= w1 < w64
    # two candidate-list entries (8 bytes each) per photon slot: per-wavefront lists and
    # the overflow list
    assert abs(Q.qed_work_bytes(1, 2000) - w1 - 16000) < 512
    # arenas: 72 bytes per photon record, 80 per pair record (a quarter of the records,
    # at least 4096), plus the count matrices, per-wavefront totals and 4 bytes per pool
    # chunk of 256 records
    a0 = Q.qed_work_bytes(1, 1000, 1 << 20)
    a1 = Q.qed_work_bytes(1, 1000, 1 << 21)
    assert a0 > w1 and abs((a1 - a0) - (72 + 20) * (1 << 20)) < 32768
    # no arenas above 1024 instances
    assert Q.qed_work_bytes(1025, 1000, 1 << 20) == Q.qed_work_bytes(1025, 1000)
    # same-step processing: per record 64 (photon) and 72 (pair) bytes more, and a second
    # set of arenas
    s0 = Q.qed_work_bytes(1, 1000, 1 << 20, True)
    s1 = Q.qed_work_bytes(1, 1000, 1 << 21, True)
    assert abs((s1 - s0) - 2 * (136 + 152 // 4) * (1 << 20)) < 65536
    assert Q.qed_work_bytes(1, 1000, 0, True) == Q.qed_work_bytes(1, 1000)
    assert Q.lib().qed_status_string(1) == b"invalid argument"
    # thinning: per-instance plan and partial sums plus a 4-byte hole list per slot
    t1, t2 = Q.qed_thin_work_bytes(1, 1000), Q.qed_thin_work_bytes(1, 2000)
    assert t1 > 0 and abs((t2 - t1) - 4000) < 512
    assert Q.qed_thin_work_bytes(0, 10) == 0 and Q.qed_thin_work_bytes(1, -1) == 0


def test_thin_argument_validation_without_device(Q):
    L = Q.lib()
    st = Q.qed_stores()
    fake = C.c_void_p(4096)
    assert L.qed_thin(None, 2, 10, 5, fake, fake, fake, 1 << 20, None) == Q.QED_ERR_ARG
    st.n_instances = 1
    st.d_instances = 4096
    st.slots[2] = 1000
    # bad species, trigger, target; too small a workspace; store columns missing
    assert L.qed_thin(C.byref(st), 3, 10, 5, fake, fake, fake, 1 << 20, None) == Q.QED_ERR_ARG
    assert L.qed_thin(C.byref(st), 2, -1, 5, fake, fake, fake, 1 << 20, None) == Q.QED_ERR_ARG
    assert L.qed_thin(C.byref(st), 2, 10, 0, fake, fake, fake, 1 << 20, None) == Q.QED_ERR_ARG
    assert L.qed_thin(C.byref(st), 2, 10, 5, fake, fake, fake, 16, None) == Q.QED_ERR_ARG
    assert L.qed_thin(C.byref(st), 2, 10, 5, fake, fake, fake, 1 << 20, None) == Q.QED_ERR_ARG
    st.slots[2] = 1 << 32
    assert L.qed_thin(C.byref(st), 2, 10, 5, fake, fake, fake, 1 << 40,
                      None) == Q.QED_ERR_UNSUPPORTED


def test_schwinger_argument_validation_without_device(Q):
    L = Q.lib()
    st = Q.qed_stores()
    st.n_instances = 1
    st.d_instances = 4096
    fake = C.c_void_p(4096)
    f = Q.qed_field()
    f.kind = Q.QED_FIELD_UNIFORM
    assert L.qed_schwinger(C.byref(st), C.byref(f), 1.0, 1.0, 1.0, fake, fake,
                           None) == Q.QED_ERR_ARG  # not a grid
    f.kind = Q.QED_FIELD_YEE
    for c in range(6):
        f.grid[c] = C.cast(C.c_void_p(4096), Q._fp)
    f.n = (C.c_int * 3)(4, 4, 4)
    f.dx = (C.c_double * 3)(1.0, 1.0, 1.0)
    assert L.qed_schwinger(C.byref(st), C.byref(f), 0.0, 1.0, 1.0, fake, fake,
                           None) == Q.QED_ERR_ARG  # dt
    assert L.qed_schwinger(C.byref(st), C.byref(f), 1.0, 1.0, 1.0, fake, fake,
                           None) == Q.QED_ERR_ARG  # lepton columns missing
    f.n = (C.c_int * 3)(2048, 2048, 1024)
    assert L.qed_schwinger(C.byref(st), C.byref(f), 1.0, 1.0, 1.0, fake, fake,
                           None) == Q.QED_ERR_ARG  # 2^32 cells


def test_generator_trials_validation_without_device(Q):
    L = Q.lib()
    tab = C.c_void_p(4096)
    out = C.c_void_p(8192)
    ok = dict(chi=1.0, gamma=100.0, dtfac=31.25, dmin=1e-3)

    def call(gen=Q.QED_GEN_MODIFIED, chi=1.0, gamma=100.0, dtfac=31.25, dmin=1e-3, first=0,
             n=10, d_out=out, work=None, wb=0, tables=tab):
        return L.qed_generator_trials(tables, gen, chi, gamma, dtfac, dmin, 5, first, n, d_out,
                                      work, wb, None)

    assert call(tables=None) == Q.QED_ERR_ARG
    assert call(tables=C.c_void_p(4100)) == Q.QED_ERR_ARG  # misaligned
    assert call(gen=3) == Q.QED_ERR_ARG
    assert call(n=-1) == Q.QED_ERR_ARG and call(first=-1) == Q.QED_ERR_ARG
    assert call(first=(1 << 63) - 5, n=10) == Q.QED_ERR_ARG  # trial index overflows
    assert call(d_out=None) == Q.QED_ERR_ARG
    assert call(chi=0.0) == Q.QED_ERR_ARG and call(gamma=0.5) == Q.QED_ERR_ARG
    assert call(dtfac=-1.0) == Q.QED_ERR_ARG and call(chi=float("nan")) == Q.QED_ERR_ARG
    need = Q.qed_generator_work_bytes(Q.QED_GEN_STANDARD, ok["chi"], ok["dmin"])
    # panels from z(1e-3) = 2^-10.5 to 2^7, 4095 / 27 per octave, plus W's n + 1 ends
    panels = math.ceil((7 - math.log2((2 / 3) * 1e-3 / 0.999)) * 4095 / 27)
    assert abs(need - 16 * panels) < 600
    assert Q.qed_generator_work_bytes(Q.QED_GEN_MODIFIED, 1.0, 1e-3) == 0
    assert Q.qed_generator_work_bytes(Q.QED_GEN_STANDARD, 1.0, 0.0) == 0
    assert Q.qed_generator_work_bytes(Q.QED_GEN_STANDARD, 1.0, 1.0) == 0
    assert Q.qed_generator_work_bytes(Q.QED_GEN_STANDARD, -1.0, 1e-3) == 0
    w = C.c_void_p(1 << 20)
    assert call(gen=Q.QED_GEN_STANDARD, work=None, wb=need) == Q.QED_ERR_ARG
    assert call(gen=Q.QED_GEN_STANDARD, work=w, wb=need - 8) == Q.QED_ERR_ARG
    assert call(gen=Q.QED_GEN_STANDARD, work=C.c_void_p((1 << 20) + 8), wb=need) == \
        Q.QED_ERR_ARG
    assert call(gen=Q.QED_GEN_STANDARD, dmin=0.0, work=w, wb=need) == Q.QED_ERR_ARG


def test_standard_w_table_validation_without_device(Q):
    L = Q.lib()
    tab, out = C.c_void_p(4096), C.c_void_p(8192)
    ok = (tab, 1e-3, 1e3, 41, 1e-3, out, None)
    for i, bad in ((0, None), (0, C.c_void_p(4100)), (5, None), (3, 0), (3, 65536),
                   (1, 0.0), (1, -1.0), (2, 1e-4), (2, float("inf")), (4, 0.0), (4, 1.0)):
        args = list(ok)
        args[i] = bad
        assert L.qed_standard_w_table(*args) == Q.QED_ERR_ARG, (i, bad)


def test_argument_validation_without_device(Q):
    L = Q.lib()
    assert L.qed_build_tables(None, 0, None) == Q.QED_ERR_ARG
    assert L.qed_build_tables(C.c_void_p(256), 16, None) == Q.QED_ERR_ARG  # too small
    assert L.qed_build_tables(C.c_void_p(8), 1 << 20, None) == Q.QED_ERR_ARG  # misaligned
    st = Q.qed_stores()
    f = Q.qed_field()
    p = Q.qed_params()
    # null everything
    assert L.qed_step(None, C.byref(st), C.byref(f), C.byref(p), None, None, None, 0,
                      None) == Q.QED_ERR_ARG
    # no instances
    fake = C.c_void_p(4096)
    assert L.qed_step(fake, C.byref(st), C.byref(f), C.byref(p), fake, fake, fake, 1 << 20,
                      None) == Q.QED_ERR_ARG
    assert L.qed_append_stats(None, None, 0, None, None) == Q.QED_ERR_ARG
    assert L.qed_photon_spectrum(C.byref(st), 1.0, 0.5, 10, fake, None) == Q.QED_ERR_ARG
