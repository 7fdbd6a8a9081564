"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host logic (DVM solver, parameters, validation)
matches what the paper fixes."""
import ctypes
import math
import re
from pathlib import Path

import numpy as np
import pytest

from paper_1510_08886_amd import lbm
from tests.golden.tables import load_dvm_tables

ROOT = Path(__file__).resolve().parent.parent


def test_library_exports_every_declared_symbol():
    header = (ROOT / "include" / "lbmdvm.h").read_text()
    names = set(re.findall(r"^\s*(?:int|const char \*)\s*(lbm_\w+)\s*\(", header, re.M))
    assert len(names) >= 16
    so = lbm.lib()
    missing = [n for n in sorted(names) if not hasattr(so, n)]
    assert not missing, missing


@pytest.mark.parametrize("m", [t for t in load_dvm_tables() if t["kind"] == "minimal"],
                         ids=lambda t: t["label"])
def test_library_solver_reproduces_printed_tables(m):
    c, w, V = lbm.Dvm.solve_weights(m["D"], m["gens"], m["Q"], m["c"] * 0.97, m["c"] * 1.03)
    assert V == m["V"]
    assert abs(c - m["c"]) <= 2e-15 * m["c"]
    for got, want in zip(w, m["weights"]):
        assert abs(got - want) <= 4e-15 * want


def test_library_solver_picks_positive_root_and_matches_oracle():
    from oracle import dvm as odvm
    for name, spec in lbm.NAMED_DVMS.items():
        c, w, V = lbm.Dvm.solve_weights(spec["dim"], spec["gens"], spec["Q"])
        if name in odvm.NAMED:
            o = odvm.named_dvm(name)
        else:
            o = odvm.solve_dvm(spec["dim"], spec["gens"], spec["Q"])
        assert abs(c - o.c) <= 2e-15 * o.c
        np.testing.assert_allclose(w, o.group_weights, rtol=4e-15)


def test_dvm_create_rejects_non_quadrature():
    spec = lbm.NAMED_DVMS["D2V17"]
    c, w, _ = lbm.Dvm.solve_weights(spec["dim"], spec["gens"], spec["Q"])
    w2 = w.copy()
    w2[1] *= 1.0 + 1e-6
    with pytest.raises(lbm.LbmError) as e:
        lbm.Dvm(2, spec["gens"], w2, c, 7)
    assert e.value.code == -4
    # exact to degree 7 is not exact to degree 9
    with pytest.raises(lbm.LbmError):
        lbm.Dvm(2, spec["gens"], w, c, 9)


def test_dvm_order_rest_then_pairs():
    d = lbm.Dvm.named("D2V37")
    v = d.velocities
    assert d.V == 37 and tuple(v[0]) == (0, 0)
    for p in range(18):
        assert tuple(v[1 + 2 * p]) == tuple(-v[2 + 2 * p])
    assert abs(d.weights.sum() - 1) < 1e-15


def test_params_match_paper_relations():
    from oracle import stepper
    from oracle import dvm as odvm
    for name, ny, kn in (("D2V17", 40, 0.1), ("D2V37", 512, 0.05), ("D3V39", 256, 0.1)):
        d = lbm.Dvm.named(name)
        spec = lbm.NAMED_DVMS[name]
        p = lbm.params(d, lbm.Problem(dim=spec["dim"], nx=1, ny=ny, nz=ny, kn=kn,
                                      hermite_order=spec["N"]))
        o = stepper.Params(odvm.named_dvm(name).c, ny, kn, 1e-3)
        assert abs(p.tau - o.tau) < 1e-16 and abs(p.tau - kn * math.sqrt(2 / math.pi)) < 1e-16
        assert abs(p.dt - o.dt) < 1e-17
        assert abs(p.omega - o.omega) < 1e-15
        assert abs(p.omega * (p.tau + p.dt / 2) - p.dt) < 1e-17
        assert abs(p.g[0] - o.g[0]) < 1e-18
        assert abs(p.u_c - 1e-3) < 1e-15
        assert abs(p.mdot_scale - 1 / (4e-3 * kn)) < 1e-9
        assert p.halo == 3


@pytest.mark.parametrize("field,value,code", [
    ("ny", 2, -1), ("hermite_order", 1, -1), ("hermite_order", 5, -1), ("kn", 0.0, -1),
    ("g", (1e-3, 1e-4), -1), ("accommodation", 1.5, -1), ("accommodation", -0.1, -1),
    ("rho0", 0.0, -1), ("nx", 0, -1), ("layout", "other", None),
])
def test_validation_errors(field, value, code):
    d = lbm.Dvm.named("D2V17")
    prob = lbm.Problem(dim=2, nx=4, ny=10, kn=0.1, hermite_order=3)
    setattr(prob, field, value)
    if code is None:     # rejected by the binding before the library
        with pytest.raises(KeyError):
            lbm.state_bytes(d, prob)
        return
    with pytest.raises(lbm.LbmError) as e:
        lbm.state_bytes(d, prob)
    assert e.value.code == code


def test_accommodation_below_one_is_2d_only():
    """Maxwell accommodation alpha < 1 (specular reflection of the rest) is
    implemented for channels; ducts and the batched engine refuse it."""
    d2 = lbm.Dvm.named("D2V17")
    lbm.state_bytes(d2, lbm.Problem(dim=2, nx=4, ny=10, kn=0.1, hermite_order=3,
                                    accommodation=0.5))
    d3 = lbm.Dvm.named("D3V39")
    with pytest.raises(lbm.LbmError) as e:
        lbm.state_bytes(d3, lbm.Problem(dim=3, nx=4, ny=10, nz=10, kn=0.1, hermite_order=3,
                                        accommodation=0.5))
    assert e.value.code == -2
    # specular partners belong to other nodes: ping-pong only (two copies)
    prob = lbm.Problem(dim=2, nx=4, ny=10, kn=0.1, hermite_order=3, accommodation=0.5)
    assert lbm.state_bytes(d2, prob)[0] == 2 * lbm.state_bytes(
        d2, lbm.Problem(dim=2, nx=4, ny=10, kn=0.1, hermite_order=3))[0]
    prob.layout = "in_place"
    with pytest.raises(lbm.LbmError) as e:
        lbm.state_bytes(d2, prob)
    assert e.value.code == -2


def test_layout_choice_sets_copies():
    d = lbm.Dvm.named("D2V37")
    base = dict(dim=2, nx=128, ny=20, kn=0.05, hermite_order=4, storage="f32")
    one = 37 * 128 * 20 * 4
    assert lbm.state_bytes(d, lbm.Problem(**base))[0] == one
    assert lbm.state_bytes(d, lbm.Problem(**base, layout="in_place"))[0] == one
    assert lbm.state_bytes(d, lbm.Problem(**base, layout="ping_pong"))[0] == 2 * one


def test_state_bytes_layout():
    d = lbm.Dvm.named("D2V37")
    one = 37 * 2048 * 512 * 4
    pop, scr = lbm.state_bytes(d, lbm.Problem(dim=2, nx=2048, ny=512, kn=0.05, hermite_order=4,
                                              storage="f32"))
    assert pop == 2 * one            # two copies, stepped two steps per launch
    assert scr < 1 << 20
    pop16, _ = lbm.state_bytes(d, lbm.Problem(dim=2, nx=2048, ny=512, kn=0.05, hermite_order=4,
                                              storage="f16dev"))
    assert pop16 == one // 2         # one array of 2-byte deviations, in place
    pop_sr, _ = lbm.state_bytes(d, lbm.Problem(dim=2, nx=2048, ny=512, kn=0.05, hermite_order=4,
                                               storage="f32sr"))
    assert pop_sr == one             # the same FP32 deviations, collided in FP64, in place


def test_unknown_storage_is_refused():
    d = lbm.Dvm.named("D2V37")
    pc = lbm.Problem(dim=2, nx=16, ny=8, kn=0.1, hermite_order=4).to_c()
    pc.storage = 5
    pop, scr = ctypes.c_size_t(), ctypes.c_size_t()
    assert lbm.lib().lbm_state_bytes(d._h, ctypes.byref(pc), ctypes.byref(pop), ctypes.byref(scr)) == -1


def test_state_bytes_in_place_up_to_512_mib_then_two_copies():
    """One population array (stepped in place) while a copy is at most 512 MiB,
    two copies (ping-pong) above: the 128 x 256 x 256 D3V39 FP32 duct needs two
    1.3 GB copies. 2D problems in FP32 deviations or FP64 with a two-step
    kernel take two copies from 64 MiB per copy: the 1024 x 256 D2V37 FP32
    channel (39 MB) one array, the 2048 x 256 one (78 MB) two copies, and so
    the FP64 1024 x 256 one; D2V32 (no two-step kernel) stays in place."""
    d2 = lbm.Dvm.named("D2V37")
    for nx, ny, st, size, copies in [(1024, 256, "f32", 4, 1), (2048, 256, "f32", 4, 2),
                                     (1024, 256, "f64", 8, 2), (1024, 128, "f64", 8, 1),
                                     (2048, 512, "f16dev", 2, 1), (2048, 512, "f32raw", 4, 1)]:
        pop, _ = lbm.state_bytes(d2, lbm.Problem(dim=2, nx=nx, ny=ny, kn=0.05, hermite_order=4,
                                                 storage=st))
        assert pop == copies * 37 * nx * ny * size, (nx, ny, st)
    d32 = lbm.Dvm.named("D2V32")
    pop, _ = lbm.state_bytes(d32, lbm.Problem(dim=2, nx=2048, ny=512, kn=0.05, hermite_order=4,
                                              storage="f32"))
    assert pop == 32 * 2048 * 512 * 4
    d3 = lbm.Dvm.named("D3V39")
    one = 39 * 128 * 256 * 256 * 4
    pop3, _ = lbm.state_bytes(d3, lbm.Problem(dim=3, nx=128, ny=256, nz=256, kn=0.1,
                                              hermite_order=3, storage="f32"))
    assert pop3 == 2 * one
    # just below the threshold: one copy
    pop4, _ = lbm.state_bytes(d3, lbm.Problem(dim=3, nx=64, ny=160, nz=160, kn=0.1,
                                              hermite_order=3, storage="f64"))
    assert pop4 == 39 * 64 * 160 * 160 * 8 and pop4 <= 512 << 20


def test_stream_copy_rejects_bad_arguments_without_a_launch():
    so = lbm.lib()
    assert so.lbm_stream_copy(None, None, 16, None) == -1
    # 16-byte alignment and size (checked before any device call)
    assert so.lbm_stream_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), 24, None) == -1
    assert so.lbm_stream_copy(ctypes.c_void_p(8), ctypes.c_void_p(32), 32, None) == -1


def test_set_graph_steps_rejects_bad_arguments():
    so = lbm.lib()
    assert so.lbm_solver_set_graph_steps(None, 4) == -1


def test_problems_beyond_32_bit_indices_are_refused():
    """Kernels index populations with 32-bit integers: V x nodes must stay below
    2^32 (a 128 x 1024 x 1024 D3V39 duct would not)."""
    d = lbm.Dvm.named("D3V39")
    with pytest.raises(lbm.LbmError) as e:
        lbm.state_bytes(d, lbm.Problem(dim=3, nx=128, ny=1024, nz=1024, kn=0.1, hermite_order=3,
                                       storage="f32"))
    assert e.value.code == -2
    pop, _ = lbm.state_bytes(d, lbm.Problem(dim=3, nx=128, ny=512, nz=1024, kn=0.1,
                                            hermite_order=3, storage="f16dev"))
    assert pop == 2 * 39 * 128 * 512 * 1024 * 2


def test_struct_layouts_match_header(tmp_path):
    """Every public struct of the header has the size and field offsets that
    the Python binding's ctypes mirror assumes (checked with gcc against the
    header itself)."""
    import ctypes
    import subprocess

    from paper_1510_08886_amd import lbm
    pairs = {"lbm_problem_t": lbm.ProblemC, "lbm_params_t": lbm.ParamsC,
             "lbm_result_t": lbm.ResultC, "lbm_wall_report_t": lbm.WallReportC,
             "lbm_dvm_model_t": lbm.DvmModelC, "lbm_profile_stats_t": lbm.ProfileStatsC,
             "lbm_batch_tuning_t": lbm.BatchTuningC, "lbm_batch_stats_t": lbm.BatchStatsC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbmdvm.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", str(ROOT / "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
