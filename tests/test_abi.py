"""C-ABI checks that need no GPU: the library loads, exports every function include/qsim.h
declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1412_2293_amd as q
from workloads import grover, qft, random_layers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qsim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    L = q.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_struct_sizes_match_header_layout():
    # qs_gate: 4 int32 + 2 uint32 + double + 2 uint64 + 32 doubles
    assert ctypes.sizeof(q.Gate) == 16 + 8 + 8 + 16 + 256
    assert ctypes.sizeof(q.Noise) == 8 + 8 + 4 + 4 + 8
    assert ctypes.sizeof(q.Plan) == 20


def _c_layout(structs):
    """sizeof and offsetof of each struct field as the C compiler lays them out from qsim.h."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qsim.h"', "int main(void) {"]
    for cname, py in structs:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0; }"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.check_output([exe]).decode()
    return dict(ln.split() for ln in out.splitlines())


def test_every_struct_matches_the_c_layout():
    structs = [("qs_gate", q.Gate), ("qs_noise", q.Noise), ("qs_plan", q.Plan),
               ("qs_srv_config", q.SrvConfig), ("qs_srv_job_info", q.SrvJobInfo), ("qs_srv_stats", q.SrvStats)]
    c = _c_layout(structs)
    for cname, py in structs:
        assert int(c[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(c[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_server_rejects_bad_config_before_device_work():
    L = q.lib()
    h = ctypes.c_void_p()
    cfg = q.SrvConfig()
    cfg.dtype, cfg.max_inflight = q.C64, 4
    assert L.qs_srv_create(ctypes.byref(cfg), None, 1 << 20, ctypes.byref(h)) == -1
    cfg.max_inflight = 0
    assert L.qs_srv_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 20), 1 << 20, ctypes.byref(h)) == -1
    cfg.max_inflight, cfg.dtype = 4, 7
    assert L.qs_srv_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 20), 1 << 20, ctypes.byref(h)) == -1
    cfg.dtype, cfg.max_chunk_traj = q.C64, 5000
    assert L.qs_srv_create(ctypes.byref(cfg), ctypes.c_void_p(1 << 20), 1 << 20, ctypes.byref(h)) == -1
    cfg.max_chunk_traj = 0
    assert L.qs_srv_create(ctypes.byref(cfg), ctypes.c_void_p((1 << 20) + 8), 1 << 20, ctypes.byref(h)) == -1
    assert "aligned" in L.qs_last_error().decode()
    jid = ctypes.c_uint64()
    assert L.qs_srv_submit(None, None, 0, 4, 0, None, 4, -1, ctypes.byref(jid)) == -1
    assert L.qs_srv_destroy(None) == 0


def test_bytes_required_rejects_bad_sizes():
    assert q.sv_bytes_required(0, q.C128, 1) == 0
    assert q.sv_bytes_required(35, q.C128, 1) == 0
    assert q.sv_bytes_required(10, 7, 1) == 0
    assert q.sv_bytes_required(10, q.C64, 0) == 0
    assert q.sv_bytes_required(10, q.C64, 3) == 3 * 1024 * 8
    assert q.fr_bytes_required(10, 9, q.C64) == 0
    assert q.fr_bytes_required(10, 8, q.C128) == 8 * 1024 * 16


def _run(gates, n, **kw):
    L = q.lib()
    ga = q.gate_array(gates)
    F = np.zeros(4)
    args = dict(init=0, dtype=q.C128, nz=None, T=4, marked=-1, plan=None, buf=None, nbytes=0)
    args.update(kw)
    return L.qs_run_trajectories(ga, len(gates), n, args["init"], args["dtype"], args["nz"], args["T"],
                                 args["marked"], args["plan"], args["buf"], args["nbytes"], None,
                                 F.ctypes.data_as(ctypes.c_void_p), None, None, None)


def test_run_trajectories_validates_before_any_device_work():
    c = grover(4, seed=0)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    assert _run(c.gates, 4, buf=None) == -1                      # NULL buffer
    assert _run(c.gates, 4, buf=fake, nbytes=16) == -1           # too small
    assert b"too small" in q.lib().qs_last_error()
    assert _run(c.gates, 0, buf=fake, nbytes=1 << 30) == -1      # n out of range
    assert _run(c.gates, 4, buf=fake, nbytes=1 << 30, init=16) == -1
    assert _run(c.gates, 4, buf=fake, nbytes=1 << 30, T=0) == -1
    bad = grover(4, seed=0)
    bad.gates[3].q0 = 9
    assert _run(bad.gates, 4, buf=fake, nbytes=1 << 30) == -1
    assert b"gate 3" in q.lib().qs_last_error()
    bad = qft(4, seed=0)
    bad.gates[1].q1 = bad.gates[1].q0
    assert _run(bad.gates, 4, buf=fake, nbytes=1 << 30) == -1
    for bad_plan in (q.Plan(fuse=1, tile_bits=16, reg_bits=4, run_bits=0),
                     q.Plan(fuse=1, tile_bits=12, reg_bits=5, run_bits=0),
                     q.Plan(fuse=2, tile_bits=0, reg_bits=0, run_bits=0)):
        assert _run(c.gates, 4, buf=fake, nbytes=1 << 30, plan=ctypes.byref(bad_plan)) == -1
    assert _run(c.gates, 4, buf=ctypes.c_void_p((1 << 20) + 8), nbytes=1 << 30) == -1   # misaligned


def test_traj_bytes_required_covers_states_and_program():
    c = qft(12, seed=0)
    for dt, s in ((q.C64, 8), (q.C128, 16)):
        for fuse in (0, 1):
            need = q.traj_bytes_required(c.gates, 12, dt, 5, plan={"fuse": fuse})
            assert need >= 6 * (1 << 12) * s


def test_handles_reject_bad_arguments():
    L = q.lib()
    h = ctypes.c_void_p()
    assert L.qs_sv_create(10, q.C128, 1, None, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.qs_sv_create(10, q.C128, 1, ctypes.c_void_p(1 << 20), 16, None, ctypes.byref(h)) == -1
    assert L.qs_fr_create(10, 0, q.C128, ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h)) == -1
    assert L.qs_copy(None, None, 16, None) == -1
    assert L.qs_apply_gate(None, None, None) == -1
    assert q.lib().qs_last_error() != b""


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import importlib
    import paper_1412_2293_amd.qsim as qm
    monkeypatch.setattr(qm, "_lib", None)
    monkeypatch.setattr(qm, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(qm.QsimError):
        qm.lib()


def test_graph_and_plan_entry_points_validate_before_device_work():
    L = q.lib()
    c = qft(10, 1)
    ga = q.gate_array(c.gates)
    h = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    # bytes_required
    assert L.qs_traj_graph_bytes_required(ga, len(ga), 10, q.C64, 4, None, ctypes.byref(sz)) == 0 and sz.value > 0
    assert L.qs_traj_graph_bytes_required(ga, len(ga), 10, q.C64, 0, None, ctypes.byref(sz)) == -1
    assert L.qs_traj_graph_bytes_required(ga, len(ga), 10, q.C64, 4, None, None) == -1
    # create: NULL out, T < 1, NULL / misaligned buffer, bad circuit, too small a buffer
    fake = ctypes.c_void_p(1 << 30)
    assert L.qs_traj_graph_create(ga, len(ga), 10, q.C64, 4, None, fake, 1 << 30, None) == -1
    assert L.qs_traj_graph_create(ga, len(ga), 10, q.C64, 0, None, fake, 1 << 30, ctypes.byref(h)) == -1
    assert L.qs_traj_graph_create(ga, len(ga), 10, q.C64, 4, None, None, 1 << 30, ctypes.byref(h)) == -1
    assert L.qs_traj_graph_create(ga, len(ga), 10, q.C64, 4, None, ctypes.c_void_p((1 << 30) + 64), 1 << 30,
                                  ctypes.byref(h)) == -1
    assert L.qs_traj_graph_create(ga, len(ga), 9, q.C64, 4, None, fake, 1 << 30, ctypes.byref(h)) == -1   # qubit 9 out of range
    assert L.qs_traj_graph_create(ga, len(ga), 10, q.C64, 4, None, fake, 1024, ctypes.byref(h)) == -1
    assert "too small" in L.qs_last_error().decode()
    F = np.zeros(4)
    assert L.qs_traj_graph_launch(None, 0, None, -1, F.ctypes.data_as(ctypes.c_void_p), None, None, None) == -1
    assert L.qs_traj_graph_destroy(None) == 0
    # plan choice
    assert L.qs_plan_choose(ga, len(ga), 10, q.C64, None, None) == -1
    p = q.Plan()
    assert L.qs_plan_choose(ga, len(ga), 35, q.C64, ctypes.byref(p), None) == -1
    assert L.qs_plan_choose(ga, len(ga), 10, 5, ctypes.byref(p), None) == -1
    assert L.qs_plan_choose(ga, len(ga), 10, q.C64, ctypes.byref(p), None) == 0 and p.fuse in (0, 1)


def test_server_calls_reject_null_handles():
    L = q.lib()
    d = ctypes.c_int()
    info = q.SrvJobInfo()
    st = q.SrvStats()
    assert L.qs_srv_poll(None, 1, ctypes.byref(d)) == -1
    assert L.qs_srv_wait(None, 1, 0.0) == -1
    assert L.qs_srv_result(None, 1, None, None, None, ctypes.byref(info)) == -1
    assert L.qs_srv_stats_get(None, ctypes.byref(st)) == -1


def test_fused_plan_limits():
    c = qft(14, 2)
    ok = {"fuse": 1, "tile_bits": 12, "reg_bits": 4, "run_bits": 5}
    assert q.traj_bytes_required(c.gates, 14, q.C64, 2, ok) > 0
    # 16-register complex<float> tiles allow at most 256 threads; complex<double> 8-register too
    assert q.traj_bytes_required(c.gates, 14, q.C64, 2, {"fuse": 1, "tile_bits": 13, "reg_bits": 4}) == 0
    assert q.traj_bytes_required(c.gates, 14, q.C128, 2, {"fuse": 1, "tile_bits": 12, "reg_bits": 3}) == 0
    assert q.traj_bytes_required(c.gates, 14, q.C128, 2, {"fuse": 1, "tile_bits": 11, "reg_bits": 3}) > 0
    # one-qubit circuits fuse into one whole-state tile
    from workloads import U1, Gate, haar_2x2
    g = [Gate(U1, q0=0, m=haar_2x2(np.random.default_rng(0)))]
    assert q.traj_bytes_required(g, 1, q.C64, 2, {"fuse": 1}) > 0


def test_size_query_is_cached_and_program_offsets_do_not_depend_on_the_batch():
    """The size query and the layout come from the run's cached preparation: repeated queries, and
    queries for other batch sizes, agree with the layout's total; the program tables' offsets
    from the first table are the same for every batch size (the run uploads them as one image
    planned once per circuit); rejected arguments still give 0."""
    c = random_layers(12, 4, seed=5, pairing="random")
    prog = ["passes", "stages", "rounds", "ops", "prefs", "jobs", "obits", "chains"]
    for dt in (q.C64, q.C128):
        for plan in (None, {"fuse": 0}, {"fuse": 1}, {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 2}):
            rel = None
            for T in (1, 5, 64, 5):
                need = q.traj_bytes_required(c.gates, 12, dt, T, plan)
                lay = q.traj_layout(c.gates, 12, dt, T, plan)
                assert need == lay["total"] > 0
                offs = [int(lay[k]) for k in prog]
                assert all(o % 256 == 0 for o in offs) and offs == sorted(offs)
                r = [o - offs[0] for o in offs]
                rel = r if rel is None else rel
                assert r == rel, (dt, plan, T)
    assert q.traj_bytes_required(c.gates, 12, q.C64, 0, None) == 0
    assert q.traj_bytes_required(c.gates, 12, q.C64, 4, {"fuse": 2}) == 0
