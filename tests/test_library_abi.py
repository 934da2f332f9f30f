"""The C-ABI library loads and exports every symbol include/airebo.h declares (CPU only)."""
import os
import re

from paper_1810_07026_amd import airebo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "airebo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(airebo_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(airebo.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = airebo.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_precision_codes_match_header():
    src = open(os.path.join(ROOT, "include", "airebo.h")).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\bAIREBO_(FP64|MIXED|SINGLE)\s*=\s*(\d+)", src))
    assert codes == {"FP64": airebo.FP64, "MIXED": airebo.MIXED, "SINGLE": airebo.SINGLE}
    assert airebo.PRECISIONS == {"fp64": airebo.FP64, "mixed": airebo.MIXED, "single": airebo.SINGLE}


def test_options_default_on_cpu():
    import ctypes
    L = airebo.load_library()
    o = airebo.Options()
    L.airebo_options_default(ctypes.byref(o))
    assert o.precision == 0 and o.term_mask == 7 and abs(o.skin - 1.0) < 1e-15
    assert L.airebo_last_error() is not None


def test_options_layout_matches_library_on_cpu():
    """The binding's Options has the C struct's size: airebo_options_default
    clears exactly sizeof(Options) bytes (the last field, schedule, included)
    and nothing beyond."""
    import ctypes
    L = airebo.load_library()
    n = ctypes.sizeof(airebo.Options)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xAB] * (n + 64)))
    L.airebo_options_default(ctypes.cast(buf, ctypes.POINTER(airebo.Options)))
    assert all(b == 0xAB for b in buf[n:])
    o = airebo.Options.from_buffer(buf)
    assert o.schedule == 0 and o.precision == 0 and o.term_mask == 7


def test_params_from_file_and_text_on_cpu():
    """The parameter set parses on the host alone, from the file and from its
    text; malformed text is rejected with the failing record named."""
    import pytest
    ps = airebo.ParamSet()
    ps.close()
    text = open(airebo.DEFAULT_PARAMS).read()
    ps = airebo.ParamSet(text=text)
    ps.close()
    bad = text.replace("tors_eps_CCCC 0.3079", "tors_eps_CCCC 0.30x9")
    assert bad != text
    with pytest.raises(airebo.AireboError) as ex:
        airebo.ParamSet(text=bad)
    assert ex.value.code == -2 and "tors_eps_CCCC" in str(ex.value)
    with pytest.raises(airebo.AireboError) as ex:
        airebo.ParamSet(text="")
    assert ex.value.code == -2
