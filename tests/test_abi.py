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


# ---------------------------------------------------------------- surrogate MLP ABI

MLP_HEADER = os.path.join(ROOT, "include", "sph_mlp.h")


def test_mlp_exports_every_declared_symbol(P):
    txt = re.sub(r"/\*.*?\*/", "", open(MLP_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(mlp_[a-z_0-9]+)\s*\(", txt)))
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", str(P.LIB_PATH)], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mlp_\w+)", out))
    assert not [n for n in names if n not in exported]
    from paper_2511_15908_amd import mlp
    assert sorted(mlp.EXPORTED) == names


def test_mlp_config_layout(P, tmp_path):
    from paper_2511_15908_amd import mlp
    src = tmp_path / "lay.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{MLP_HEADER}"', "int main(void){",
             'printf("size %zu\\n", sizeof(mlp_config));']
    for f, _ in mlp.MlpConfig._fields_:
        lines.append(f'printf("{f} %zu\\n", offsetof(mlp_config, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    assert int(got["size"]) == C.sizeof(mlp.MlpConfig)
    for f, _ in mlp.MlpConfig._fields_:
        assert int(got[f]) == getattr(mlp.MlpConfig, f).offset, f


def _mlp_cfg(**over):
    from paper_2511_15908_amd import mlp
    c = mlp.MlpConfig()
    c.abi_version, c.n_in, c.n_out, c.hidden, c.layers, c.max_batch = 1, 126, 6, 256, 3, 4096
    c.beta1, c.beta2, c.eps = 0.9, 0.999, 1e-8
    for k, v in over.items():
        if k == "reserved":
            c.reserved[0] = v
        else:
            setattr(c, k, v)
    return c


def test_mlp_validation_and_workspace(P):
    from paper_2511_15908_amd import mlp
    L = mlp.lib()
    out = C.c_size_t(0)
    assert L.mlp_workspace_size(C.byref(_mlp_cfg()), C.byref(out)) == 0
    # parameters: 128x256+256 + 2 (256x256+256) + 16x256+16; activations of 4096 rows
    assert out.value > 4 * 4 * 168720 + 4096 * 256 * 6 * 3
    # more than 128 inputs pad to 256 columns: a larger first layer
    small = out.value
    assert L.mlp_workspace_size(C.byref(_mlp_cfg(n_in=200)), C.byref(out)) == 0 and out.value > small
    for bad in [dict(n_in=0), dict(n_in=257), dict(n_out=17), dict(hidden=100), dict(hidden=512),
                dict(layers=0), dict(layers=5), dict(max_batch=0), dict(max_batch=70000), dict(beta1=1.0),
                dict(eps=0.0), dict(abi_version=2), dict(reserved=1)]:
        assert L.mlp_workspace_size(C.byref(_mlp_cfg(**bad)), C.byref(out)) == 1, bad
    ctx = C.c_void_p()
    # no workspace: rejected before any device work
    assert L.mlp_init(C.byref(_mlp_cfg()), None, 0, None, C.byref(ctx)) == 2
    assert L.mlp_destroy(None) == 0
    assert L.mlp_param_count(None) == 0
    # the stand-alone product rejects bad layouts and misaligned operands without launching
    assert L.mlp_gemm_bf16(None, 2, 0, C.c_void_p(256), 8, C.c_void_p(256), 8, 8, 8, 8, C.c_void_p(256), 8) == 1
    assert L.mlp_gemm_bf16(None, 0, 0, C.c_void_p(258), 8, C.c_void_p(256), 8, 8, 8, 8, C.c_void_p(256), 8) == 1
    assert L.mlp_gemm_bf16(None, 0, 0, C.c_void_p(256), 4, C.c_void_p(256), 8, 8, 8, 8, C.c_void_p(256), 8) == 1
