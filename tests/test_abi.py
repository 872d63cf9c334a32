"""CPU checks of the C ABI: the library builds for gfx950, loads, exports every
entry point the header declares, and the binding's struct layouts match the C
compiler's."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpet.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:gpet_status|void|const char \*)\s*(gpet_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2603_07327_amd import gpet
    if not os.path.exists(gpet.LIB_PATH):
        from paper_2603_07327_amd import build
        build.build()
    return gpet.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2603_07327_amd import gpet
    assert sorted(gpet.EXPORTS) == names


def test_struct_layouts_match_c(tmp_path):
    """Sizes of every struct and offsets of every field (Stats: size only, its
    Python field names are short forms)."""
    from paper_2603_07327_amd import gpet
    structs = {"gpet_material": gpet.Material, "gpet_physics": gpet.Physics, "gpet_layer": gpet.Layer,
               "gpet_scanner": gpet.Scanner, "gpet_geometry_info": gpet.GeometryInfo,
               "gpet_phantom": gpet.Phantom, "gpet_source": gpet.Source, "gpet_hits": gpet.Hits,
               "gpet_stats": gpet.Stats, "gpet_digitizer": gpet.Digitizer, "gpet_singles": gpet.Singles,
               "gpet_surrogate_spec": gpet.SurrogateSpec,
               "gpet_coincidences": gpet.Coincidences, "gpet_tallies": gpet.Tallies,
               "gpet_instance": gpet.Instance}
    src = tmp_path / "probe.c"
    lines = [f'printf("{k} %zu\\n", sizeof({k}));' for k in structs]
    for k, cls in structs.items():
        if cls is gpet.Stats:
            continue
        for f, _ in cls._fields_:
            lines.append(f'printf("{k}.{f} %zu\\n", offsetof({k}, {f}));')
    body = "\n".join(lines)
    src.write_text(f'#include <stddef.h>\n#include <stdio.h>\n#include "{HEADER}"\nint main(void){{{body} return 0;}}\n')
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    sizes = dict(ln.split() for ln in out if ln)
    for k, cls in structs.items():
        assert int(sizes[k]) == ctypes.sizeof(cls), k
        if cls is gpet.Stats:
            continue
        for f, _ in cls._fields_:
            assert int(sizes[f"{k}.{f}"]) == getattr(cls, f).offset, f"{k}.{f}"


def test_context_requires_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2603_07327_amd.gpet import Context
    with pytest.raises(RuntimeError):
        Context(0)
