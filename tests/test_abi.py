"""The C ABI of libsph.so without a GPU: the library loads, exports every
entry point include/sph.h declares, its structs have the layout the binding
assumes, and host-side validation rejects bad input before any device work."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


@pytest.fixture(scope="module")
def P():
    import paper_2511_15908_amd as P
    P.load_library()
    return P


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(P):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", str(P.LIB_PATH)], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (sph_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    from paper_2511_15908_amd import _binding
    assert sorted(_binding.EXPORTED) == names


def test_struct_layout_matches_header(P, tmp_path):
    from paper_2511_15908_amd import _binding as B
    src = tmp_path / "lay.c"
    fields = {"sph_params": B.SphParams, "sph_scene": B.SphScene, "sph_info": B.SphInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    for cname, cls in fields.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def _scene():
    from paper_2511_15908_amd import scenes
    return scenes.small_scene(seed=3, nf=(4, 4, 4), n_tank=(8, 6, 6))


def _ws(P, sc, **over):
    from paper_2511_15908_amd import _binding as B
    L = P.load_library()
    pr = dict(sc.params)
    prec = over.pop("precision", sc.precision)
    vmax = over.pop("v_max", 0.0)
    pr.update({k: v for k, v in over.items() if k in pr})
    Pm = B.make_params(pr, prec, vmax)
    for k, v in over.items():
        if k not in pr:
            setattr(Pm, k, v)
    A = B._SceneArrays(sc)
    out = C.c_size_t(0)
    return L.sph_workspace_size(C.byref(Pm), C.byref(A.struct), C.byref(out)), out.value


def test_workspace_size_valid(P):
    st, nb = _ws(P, _scene())
    assert st == 0 and nb > 0
    st64, nb64 = _ws(P, _scene(), precision="f64")
    assert st64 == 0 and nb64 > nb


@pytest.mark.parametrize("over,code", [
    ({"h": -1.0}, 1), ({"h": 0.0}, 1), ({"dt": 0.0}, 1), ({"rho0": float("nan")}, 1),
    ({"nu": -1.0}, 1), ({"smoothing_window": 0}, 1), ({"abi_version": 7}, 1), ({"flags": 64}, 6),
    ({"domain_hi": (0.0, 0.0, 0.0), "domain_lo": (1.0, 1.0, 1.0)}, 1), ({"h": 1e-6}, 6),
    ({"v_max": -1.0}, 1),
])
def test_workspace_size_rejects_params(P, over, code):
    st, _ = _ws(P, _scene(), **over)
    assert st == code


def test_workspace_rejects_bad_scene(P):
    sc = _scene()
    sc.x = sc.x.copy()
    sc.x[3, 1] = np.nan
    assert _ws(P, sc)[0] == 1
    sc = _scene()
    sc.object = sc.object.copy()
    sc.object[sc.type == 2][:1] = 9
    idx = np.nonzero(sc.type == 2)[0][0]
    sc.object[idx] = 9
    assert _ws(P, sc)[0] == 1
    sc = _scene()
    sc.spring_ij = sc.spring_ij.copy()
    sc.spring_ij[0, 0] = 0            # a fluid particle
    assert _ws(P, sc)[0] == 1
    sc = _scene()
    sc.mass = sc.mass.copy()
    sc.mass[0] = 0.0
    assert _ws(P, sc)[0] == 1
    sc = _scene()
    sc.object_pose0 = sc.object_pose0.copy()
    sc.object_pose0[1, 3:] = 0.0
    assert _ws(P, sc)[0] == 1


def test_init_rejects_missing_or_misaligned_workspace(P):
    from paper_2511_15908_amd import _binding as B
    L = P.load_library()
    sc = _scene()
    Pm = B.make_params(sc.params, sc.precision)
    A = B._SceneArrays(sc)
    ctx = C.c_void_p()
    assert L.sph_init(C.byref(Pm), C.byref(A.struct), None, 1 << 30, None, C.byref(ctx)) == 2
    assert L.sph_init(C.byref(Pm), C.byref(A.struct), C.c_void_p(0x1000), 16, None, C.byref(ctx)) == 2
    assert L.sph_init(C.byref(Pm), C.byref(A.struct), C.c_void_p(0x1001), 1 << 40, None, C.byref(ctx)) == 2
    assert not ctx.value


def test_null_context_calls(P):
    L = P.load_library()
    d = (C.c_double * 3)()
    assert L.sph_step(None, 1, None) == 1
    assert L.sph_get_body_wrench(None, 0, d, d, 0) == 1
    assert L.sph_destroy(None) == 0
    assert L.sph_status_string(5) == b"simulation became unstable"
    assert L.sph_last_error(None) == b"null context"
    assert L.sph_profile_phase_name(5) == b"density"
