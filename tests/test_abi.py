"""CPU checks of the C-ABI boundary: the built library loads, exports every function that
include/ipgc.h declares, the Python mirrors of the structs match the header, and the product
package does not reach the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipgc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ipgc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1912_01478_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1912_01478_amd import build
        build.build()
    return pkg.library()


def test_header_declares_entry_points():
    names = declared_functions()
    assert "ipgc_color_graph" in names and "ipgc_color_graph_ex" in names
    import paper_1912_01478_amd as pkg
    assert sorted(pkg.EXPORTS) == names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert getattr(lib, name) is not None


def test_version(lib):
    assert lib.ipgc_version() >> 16 == 2


# Structs the binding mirrors, with the fields whose offsets are compared against the header.
MIRRORS = {
    "ipgc_options": ("Options", ["threshold", "light_max_degree", "hub_min_degree", "validate", "flags", "profile",
                                 "workgroups", "tail_workgroups", "barrier_timeout_ms", "reserved"]),
    "ipgc_trace": ("Trace", ["capacity", "wl_size", "wl_degree", "topology", "recorded", "topo_graphs"]),
    "ipgc_profile": ("Profile", ["mask", "kinds", "ms", "launches", "unit_kinds", "reserved", "units", "phase_ticks",
                                 "phase_capacity", "phase_recorded", "tick_khz"]),
    "ipgc_server_config": ("ServerConfig", ["node_capacity", "edge_capacity", "max_jobs", "rounds_per_step", "mode",
                                            "reserved", "options"]),
    "ipgc_job_result": ("JobResult", ["job_id", "status", "rounds"]),
    "ipgc_server_stats": ("ServerStats", ["steps", "cancelled", "rounds", "submitted", "admitted", "completed",
                                          "resident", "queued", "resident_nodes", "resident_edges", "peak_resident",
                                          "arena_bytes", "units"]),
}


@pytest.fixture(scope="module")
def c_layouts(tmp_path_factory):
    """sizeof and offsetof of every mirrored struct, as a C compiler lays out include/ipgc.h."""
    import subprocess
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stddef.h>", "#include <stdio.h>", "#include \"ipgc.h\"", "int main(void) {"]
    for cname, (_, fields) in MIRRORS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in fields:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        out[(a, b)] = int(c)
    return out


@pytest.mark.parametrize("cname", sorted(MIRRORS))
def test_struct_layouts_match_header(c_layouts, cname):
    import paper_1912_01478_amd as pkg
    pyname, fields = MIRRORS[cname]
    cls = getattr(pkg, pyname)
    assert ctypes.sizeof(cls) == c_layouts[(cname, "size")]
    assert [f for f, _ in cls._fields_] == fields
    for f in fields:
        assert getattr(cls, f).offset == c_layouts[(cname, f)], (cname, f)


def test_flags_match_header():
    """Every IPGC_FLAG_* value of the header is the binding's FLAG_* value of the same name."""
    import re

    import paper_1912_01478_amd as pkg
    with open(os.path.join(ROOT, "include", "ipgc.h")) as f:
        flags = dict(re.findall(r"IPGC_FLAG_(\w+) = (\d+)", f.read()))
    assert set(flags) == {"STEPPED", "LIGHT_PULL", "LIGHT_PUSH", "RACY", "PER_GRAPH"}
    for name, value in flags.items():
        assert getattr(pkg, "FLAG_" + name) == int(value), name


def test_kernel_names(lib):
    names = []
    k = 0
    while lib.ipgc_kernel_name(k):
        names.append(lib.ipgc_kernel_name(k).decode())
        k += 1
    assert len(names) >= 4 and len(set(names)) == len(names)
    assert lib.ipgc_kernel_name(-1) == b"" and lib.ipgc_kernel_name(99) == b""
    units = []
    k = 0
    while lib.ipgc_unit_name(k):
        units.append(lib.ipgc_unit_name(k).decode())
        k += 1
    assert len(units) >= 4 and len(set(units)) == len(units)


def test_product_package_does_not_import_oracle():
    pkg_dir = os.path.join(ROOT, "paper_1912_01478_amd")
    for dirpath, _, files in os.walk(pkg_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "ipgc_oracle", "libipgc_oracle"):
                    assert bad not in src, (f, bad)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_1912_01478_amd as pkg
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(ImportError):
        pkg.library()


def test_noalloc_scratch_size_matches_binding():
    import paper_1912_01478_amd as pkg
    text = open(HEADER).read()
    m = re.search(r"#define\s+IPGC_NOALLOC_SCRATCH_BYTES\s+\((\d+)ull\s*<<\s*(\d+)\)", text)
    assert m, "IPGC_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == pkg.NOALLOC_SCRATCH_BYTES
