"""The C ABI without a GPU: the header is valid C, the library loads and
exports every function the header declares, and argument validation (a pure
host step that runs before any HIP call) rejects bad configurations."""

import ctypes
import struct
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pino_[a-z0-9_]+)\s*\(", text)))


def test_headers_compile_as_c(tmp_path):
    for h in HEADERS:
        src = tmp_path / "t.c"
        src.write_text(f'#include "{h}"\nint main(void) {{ return 0; }}\n')
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-c", str(src), "-o", str(tmp_path / "t.o")],
                       check=True)


def test_library_exports_every_declared_symbol():
    import paper_2510_02873_amd as P
    L = ctypes.CDLL(P.LIB_PATH)
    names = [n for h in HEADERS for n in _declared(h)]
    assert "pino_collapse_init" in names and "pino_collapse_eval" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared but not exported"


def _cfg(P, **kw):
    a = np.geomspace(1e-3, 1.0, 16)
    return P.Config([(a, a)], **kw)


@pytest.mark.parametrize("bad", ["version", "method", "precision", "device", "nonmono", "short", "table",
                                 "surrogate_blob", "rtol_big", "rtol_nan", "rtol_negative"])
def test_init_rejects_bad_config(bad):
    import paper_2510_02873_amd as P
    a = np.geomspace(1e-3, 1.0, 16)
    if bad == "version":
        cfg = _cfg(P, abi_version=2)
    elif bad == "method":
        cfg = _cfg(P, method=7)
    elif bad == "precision":
        cfg = _cfg(P, precision=9)
    elif bad == "device":
        cfg = _cfg(P, device=-1)
    elif bad == "nonmono":
        D = a.copy()
        D[5] = D[4]
        cfg = P.Config([(a, D)])
    elif bad == "short":
        cfg = P.Config([(a[:3], a[:3])])
    elif bad == "table":
        cfg = _cfg(P, method=P.PINO_TABULATED)
    elif bad.startswith("rtol"):
        rtol = {"rtol_big": 0.5, "rtol_nan": float("nan"), "rtol_negative": -1e-7}[bad]
        # a well-formed blob (header + 8705 zero parameters), so only the
        # tolerance is at fault
        from paper_2510_02873_amd import _abi
        blob = b"PINOMLP1" + struct.pack("<ii", 1, _abi.PINO_MLP_PARAMS) + bytes(4 * _abi.PINO_MLP_PARAMS)
        cfg = _cfg(P, precision=P.PINO_SURROGATE, mlp_blob=blob, certify_rtol=rtol)
    else:
        cfg = _cfg(P, precision=P.PINO_SURROGATE, mlp_blob=b"\x00" * 16)
    with pytest.raises(P.PinoError) as e:
        P.pino_collapse_init(cfg)
    assert e.value.status == P.PINO_ERR_ARG
    assert P.pino_collapse_last_error(None)
    if bad.startswith("rtol"):
        assert "certify_rtol" in P.pino_collapse_last_error(None)


def test_init_null_and_nan():
    import paper_2510_02873_amd as P
    L = P.lib()
    out = ctypes.c_void_p()
    assert L.pino_collapse_init(None, ctypes.byref(out)) == P.PINO_ERR_ARG
    assert out.value is None
    a = np.geomspace(1e-3, 1.0, 16)
    D = a.copy()
    D[3] = np.nan
    with pytest.raises(P.PinoError):
        P.pino_collapse_init(P.Config([(a, D)]))


def test_eval_and_free_null_ctx():
    import paper_2510_02873_amd as P
    L = P.lib()
    assert L.pino_collapse_eval(None, None, 0, 0, None) == P.PINO_ERR_ARG
    assert L.pino_collapse_free(None) == P.PINO_OK


@pytest.mark.parametrize("n_side,box", [(1, 100.0), (2000, 100.0), (32, 0.0), (32, float("nan")), (32, -5.0)])
def test_field_create_rejects_bad_grid(n_side, box):
    """pino_field_create validates before any HIP call."""
    import paper_2510_02873_amd as P
    with pytest.raises(P.PinoError) as e:
        P.Field(n_side, box)
    assert e.value.status == P.PINO_ERR_ARG
    assert "n_side" in P._abi.pino_field_last_error(None)


def test_interp_calls_reject_bad_sizes():
    """The interpolation entry points validate before any HIP call."""
    import torch
    import paper_2510_02873_amd as P
    from paper_2510_02873_amd import _abi
    one = torch.zeros(1, dtype=torch.float64)
    many = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(P.PinoError) as e:
        _abi.pino_spline_eval(one, one, one, many, many)            # a single knot
    assert e.value.status == P.PINO_ERR_ARG and "2 <= n" in str(e.value)
    with pytest.raises(P.PinoError) as e:
        _abi.pino_spline_build(torch.zeros(4096, dtype=torch.float64), torch.zeros(4096, dtype=torch.float64),
                               torch.zeros(4096, dtype=torch.float64), torch.zeros(4096, dtype=torch.float64))
    assert e.value.status == P.PINO_ERR_ARG
    with pytest.raises(P.PinoError) as e:
        _abi.pino_table_build(many, torch.zeros((1, 4, 8), dtype=torch.float64), many, many)   # nx = 1
    assert e.value.status == P.PINO_ERR_ARG


def test_mlp_calls_reject_null_handle():
    """The network entry points validate their handle before any HIP call."""
    import paper_2510_02873_amd as P
    from paper_2510_02873_amd import _abi
    L = _abi._bind_mlp()
    assert L.pino_mlp_set_bf16_forward(None, 1) == P.PINO_ERR_ARG
    assert L.pino_mlp_grad(None, None, None, 16, None, None, None) == P.PINO_ERR_ARG
    assert L.pino_mlp_adam(None, None, 1e-3, 0.9, 0.999, 1e-8, None) == P.PINO_ERR_ARG
    assert L.pino_mlp_forward(None, None, None, 4, None) == P.PINO_ERR_ARG
    assert L.pino_mlp_free(None) == P.PINO_OK
