"""The C ABI library builds for gfx950, loads, and exports every entry point
that include/ecmd.h declares (no GPU call is made)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecmd.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecmd_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("ecmd_ctx_create", "ecmd_estimate_divergence", "ecmd_estimate_divergence_batched",
                 "ecmd_probe_point", "ecmd_probe_bound", "ecmd_probe_pixels", "ecmd_downsample",
                 "ecmd_cnn_forward", "ecmd_cnn_train_step", "ecmd_estimate_divergence_learned"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2209_13168_amd import ecmd

    lib = ctypes.CDLL(ecmd.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert ecmd.lib().ecmd_version().decode().startswith("ecmd")


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets that a C
    compiler gives the header's structs."""
    import subprocess

    from paper_2209_13168_amd import ecmd

    pairs = [("ecmd_sensor", ecmd.Sensor), ("ecmd_events", ecmd.EventsS), ("ecmd_window", ecmd.WindowS),
             ("ecmd_plan_info", ecmd.PlanInfo), ("ecmd_plan_limits", ecmd.PlanLimitsS),
             ("ecmd_search", ecmd.SearchS), ("ecmd_result", ecmd.ResultS), ("ecmd_profile", ecmd.ProfileS),
             ("ecmd_tuning", ecmd.TuningS)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ecmd.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["cc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for cname, py in pairs:
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
