"""Cooperative grids are sized from the registers and LDS the compiler
recorded for each kernel when the library was built (the generated
resource table).  A kernel missing from that table would be sized by a
fallback guess, so every name the sizing looks up must be there: each
one-step and two-step tile variant of the persistent, message-driven and
multi-resolution kernels, with the schedule and load-imbalance template
flags.  Host-only (reads the table the build wrote; no GPU)."""
import os
import re

import pytest

PKG = os.path.join(os.path.dirname(__file__), "..", "paper_2605_12734_amd")
TABLE = os.path.join(PKG, "_build", "kernel_resources.inc")
KERNELS = os.path.join(PKG, "csrc", "kernels.hip")


def _variants(macro):
    src = open(KERNELS).read()
    m = re.search(r"#define " + macro + r"\(X\)((?:[^\n]*\\\n)*[^\n]*)", src)
    assert m, macro
    return [(t, int(x), int(y)) for t, x, y in re.findall(r"X\((double|float), (\d+), (\d+)\)", m.group(1))]


def _table():
    if not os.path.exists(TABLE):
        pytest.skip("library not built")
    rows = {}
    for ln in open(TABLE):
        m = re.match(r'\{"([^"]+)", (\d+), (\d+), (\d+)\},', ln.strip())
        if m:
            rows[m.group(1)] = tuple(int(v) for v in m.groups()[1:])
    return rows


def test_variant_lists_parse():
    assert len(_variants("OD_VARIANTS_F64")) == 13 and len(_variants("OD_VARIANTS_F32")) == 12
    assert len(_variants("OD_VARIANTS2_F64")) == 6 and len(_variants("OD_VARIANTS2_F32")) == 3


def test_every_cooperative_kernel_recorded():
    rows = _table()
    names = []
    for t, x, y in _variants("OD_VARIANTS_F64") + _variants("OD_VARIANTS_F32"):
        for dyn in ("true", "false"):
            names.append(f"od::k_persistent<{t}, {x}, {y}, {dyn}>")
        names.append(f"od::k_msgdriven<{t}, {x}, {y}>")
        names.append(f"od::k_persistent_mr<{t}, {x}, {y}>")
    for t, x, y in _variants("OD_VARIANTS2_F64") + _variants("OD_VARIANTS2_F32"):
        for imb in ("true", "false"):
            for dyn in ("true", "false"):
                names.append(f"od::k_persistent2<{t}, {x}, {y}, {dyn}, {imb}>")
            names.append(f"od::k_msgdriven2<{t}, {x}, {y}, {imb}>")
    missing = [n for n in names if n not in rows]
    assert not missing, missing[:5]


def test_imbalance_variants_keep_lds():
    # the load-imbalance variant of a two-step kernel runs its one-step
    # re-runs in the same LDS array: its recorded LDS equals the uniform one's
    rows = _table()
    for t, x, y in _variants("OD_VARIANTS2_F64") + _variants("OD_VARIANTS2_F32"):
        for dyn in ("true", "false"):
            a = rows[f"od::k_persistent2<{t}, {x}, {y}, {dyn}, false>"]
            b = rows[f"od::k_persistent2<{t}, {x}, {y}, {dyn}, true>"]
            assert a[2] == b[2], (t, x, y, dyn)
        assert rows[f"od::k_msgdriven2<{t}, {x}, {y}, false>"][2] == rows[f"od::k_msgdriven2<{t}, {x}, {y}, true>"][2]
