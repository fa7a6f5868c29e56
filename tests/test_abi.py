"""The C ABI library without a GPU: it loads, exports what include/cc.h declares, validates
arguments, sizes workspaces, and stays independent of the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cc.h")
PKG = os.path.join(ROOT, "paper_1807_10727_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(cc_[a-z0-9_]+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("cc_create", "cc_workspace_size", "cc_set_workspace", "cc_contract_round", "cc_run",
                 "cc_labels", "cc_round_parents", "cc_destroy", "cc_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1807_10727_amd import _cc
    lib = ctypes.CDLL(_cc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    nm = subprocess.run(["nm", "-D", "--defined-only", _cc.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r"\bT (cc_[a-z0-9_]+)", nm))
    assert set(declared_functions()) <= exported


def test_binding_names_match_the_abi():
    import paper_1807_10727_amd._cc as b
    for n in declared_functions():
        if n in ("cc_kernel_family_count", "cc_kernel_family_name"):
            continue
        assert hasattr(b, n), n


def test_product_never_touches_the_oracle():
    # the library links no oracle symbol and no package source imports the oracle
    from paper_1807_10727_amd import _cc
    nm = subprocess.run(["nm", "-D", _cc.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    assert "lco_" not in nm
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "lc_oracle" not in src, f


def test_create_validates_arguments():
    from paper_1807_10727_amd import _cc
    bad = [
        dict(n_vertices=-1, n_edges=1, layout=0),
        dict(n_vertices=1 << 31, n_edges=1, layout=0),
        dict(n_vertices=10, n_edges=-1, layout=0),
        dict(n_vertices=10, n_edges=1 << 32, layout=0),
        dict(n_vertices=10, n_edges=1, layout=3),
    ]
    for kw in bad:
        with pytest.raises(_cc.CCError) as e:
            _cc.cc_create(kw["n_vertices"], kw["n_edges"], kw["layout"], 0x1000, 0x2000)
        assert e.value.status == _cc.CC_E_ARG
    with pytest.raises(_cc.CCError):
        _cc.cc_create(10, 5, _cc.CC_EDGES_SOA_I32, 0x1000, 0)     # dst missing
    with pytest.raises(_cc.CCError):
        _cc.cc_create(10, 5, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, max_rounds=-2)
    ctx = _cc.cc_create(10, 5, _cc.CC_EDGES_PACKED_U64, 0x1000, 0)   # packed: dst unused
    _cc.cc_destroy(ctx)
    ctx = _cc.cc_create(10, 0, _cc.CC_EDGES_SOA_I32, 0, 0)           # no records: no pointers needed
    _cc.cc_destroy(ctx)


def test_workspace_size_and_state_errors():
    from paper_1807_10727_amd import _cc
    sizes = {}
    for n, m in ((1, 0), (1000, 5000), (1 << 20, 1 << 22)):
        ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_ROUND0_DIRECT)
        sizes[(n, m)] = _cc.cc_workspace_size(ctx)
        if n == 1000:
            with pytest.raises(_cc.CCError) as e:
                _cc.cc_set_workspace(ctx, 0x100000, 16)
            assert e.value.status == _cc.CC_E_NOMEM
            with pytest.raises(_cc.CCError) as e:
                _cc.cc_set_workspace(ctx, 0x100001, 1 << 30)
            assert e.value.status == _cc.CC_E_ARG
            with pytest.raises(_cc.CCError) as e:
                _cc.cc_contract_round(ctx)
            assert e.value.status == _cc.CC_E_NOMEM
        _cc.cc_destroy(ctx)
    big = sizes[(1 << 20, 1 << 22)]
    # state arrays (about 38 bytes per id) and two key buffers of 8 bytes per record dominate
    assert 16 * (1 << 22) + 36 * (1 << 20) < big < 18 * (1 << 22) + 80 * (1 << 20)
    assert sizes[(1, 0)] < sizes[(1000, 5000)] < big


def test_round0_layout_flags():
    """The tiled round 0 doubles the key buffers (16 more bytes per record) and is chosen by
    default from 2^20 ids and records up to 2^26 ids; contradictory or impossible requests
    are argument errors."""
    from paper_1807_10727_amd import _cc
    n, m = 1 << 20, 1 << 22

    def size(n, m, flags):
        ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=flags)
        try:
            return _cc.cc_workspace_size(ctx)
        finally:
            _cc.cc_destroy(ctx)

    direct = size(n, m, _cc.CC_ROUND0_DIRECT)
    tiled = size(n, m, _cc.CC_ROUND0_TILED)
    assert 16 * m <= tiled - direct < 16 * m + (m // 2) * 4 + (1 << 20)
    assert size(n, m, 0) == tiled
    assert size(n - 1, m, 0) == size(n - 1, m, _cc.CC_ROUND0_DIRECT)      # below 2^20 ids
    assert size(1 << 27, m, 0) == size(1 << 27, m, _cc.CC_ROUND0_DIRECT)  # above 2^26 ids
    assert size(1000, 5000, _cc.CC_ROUND0_TILED) > size(1000, 5000, 0)
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000,
                      flags=_cc.CC_ROUND0_TILED | _cc.CC_ROUND0_DIRECT)
    assert e.value.status == _cc.CC_E_ARG
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_create((1 << 26) + 1, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_ROUND0_TILED)
    assert e.value.status == _cc.CC_E_ARG
    ctx = _cc.cc_create(1 << 26, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_ROUND0_TILED)
    _cc.cc_destroy(ctx)


def test_labels_before_run_is_a_state_error():
    from paper_1807_10727_amd import _cc
    ctx = _cc.cc_create(10, 5, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000)
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_labels(ctx, 0x3000)
    assert e.value.status == _cc.CC_E_STATE
    _cc.cc_destroy(ctx)


def test_kernel_families_listed():
    from paper_1807_10727_amd import _cc
    names = _cc.cc_kernel_family_names()
    for want in ("min1", "min2", "parent", "relabel", "sort_scatter", "unique", "compose", "part_a_hist",
                 "part_b_scatter", "part_rows_hist", "part_rows_scatter", "min1_tiled", "min2_tiled",
                 "relabel_tiled"):
        assert want in names


def test_inspection_and_checkpoint_entry_points_validate_without_a_gpu():
    """The test and inspection half of the boundary: explicit priorities, per-round parents,
    the round minima and checkpoints reject bad calls before touching the device."""
    from paper_1807_10727_amd import _cc
    for want in ("cc_set_explicit_priorities", "cc_debug_round_arrays", "cc_save_state", "cc_load_state"):
        assert want in declared_functions()
    n, m = 1000, 5000

    def size(flags):
        ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=flags)
        try:
            return _cc.cc_workspace_size(ctx)
        finally:
            _cc.cc_destroy(ctx)

    base = size(_cc.CC_ROUND0_DIRECT)
    # the inverse of an explicit table: 4 bytes per vertex; the round records: 20 bytes per vertex
    assert 4 * n <= size(_cc.CC_ROUND0_DIRECT | _cc.CC_EXPLICIT_PRIO) - base <= 4 * n + 256
    assert 20 * n <= size(_cc.CC_ROUND0_DIRECT | _cc.CC_RECORD_ROUNDS) - base <= 20 * n + 256
    # explicit priorities run round 0 directly
    assert size(_cc.CC_EXPLICIT_PRIO) == size(_cc.CC_ROUND0_DIRECT | _cc.CC_EXPLICIT_PRIO)
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_EXPLICIT_PRIO | _cc.CC_ROUND0_TILED)
    assert e.value.status == _cc.CC_E_ARG

    ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000)
    with pytest.raises(_cc.CCError) as e:     # no CC_EXPLICIT_PRIO
        _cc.cc_set_explicit_priorities(ctx, 0, 0x3000)
    assert e.value.status == _cc.CC_E_STATE
    for r in (0, -1):
        with pytest.raises(_cc.CCError) as e:   # no round has run
            _cc.cc_round_parents(ctx, r, 0x3000)
        assert e.value.status == _cc.CC_E_STATE
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_debug_round_arrays(ctx, 0x3000, 0x4000)
    assert e.value.status == _cc.CC_E_STATE
    with pytest.raises(_cc.CCError) as e:      # no workspace yet
        _cc.cc_save_state(ctx)
    assert e.value.status == _cc.CC_E_NOMEM
    with pytest.raises(_cc.CCError) as e:
        _cc.cc_load_state(ctx, b"\0" * 64)
    assert e.value.status == _cc.CC_E_NOMEM
    _cc.cc_destroy(ctx)

    ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_EXPLICIT_PRIO)
    for r, ptr in ((-1, 0x3000), (0, 0)):
        with pytest.raises(_cc.CCError) as e:
            _cc.cc_set_explicit_priorities(ctx, r, ptr)
        assert e.value.status == _cc.CC_E_ARG
    _cc.cc_set_explicit_priorities(ctx, 0, 0x3000)   # only stored: read by the rounds that use it
    _cc.cc_set_explicit_priorities(ctx, 2, 0x5000)
    _cc.cc_set_explicit_priorities(ctx, 0, 0x7000)   # replaces round 0's table
    _cc.cc_destroy(ctx)

    ctx = _cc.cc_create(n, m, _cc.CC_EDGES_SOA_I32, 0x1000, 0x2000, flags=_cc.CC_TREE)
    with pytest.raises(_cc.CCError) as e:      # the minima are LocalContraction's
        _cc.cc_debug_round_arrays(ctx, 0x3000, 0x4000)
    assert e.value.status == _cc.CC_E_STATE
    _cc.cc_destroy(ctx)


STRUCTS = ("cc_tuning", "cc_round_stats", "cc_batch_config", "cc_server_config", "cc_request_result",
           "cc_server_info_t", "cc_graph_desc", "cc_options")


def header_struct_fields(name):
    """Field names of a `typedef struct {...} name;` in include/cc.h, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", text, flags=re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "const void *src, *dst" -> src, dst; "int32_t round0" -> round0
        first, *rest = decl.split(",")
        out.append(re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*$", first)[0])
        out += [re.sub(r"[\s*]", "", r) for r in rest]
    return out


def test_marshalled_structs_match_the_header():
    """The ctypes mirrors of the structs the boundary passes by pointer have the header's
    fields in the header's order, and (compiled with the host C compiler) the same size and
    field offsets."""
    from paper_1807_10727_amd import _cc
    for name in STRUCTS:
        mirror = getattr(_cc, name)
        assert [f[0] for f in mirror._fields_] == header_struct_fields(name), name
    import shutil
    import tempfile
    if not shutil.which("gcc"):
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#include \"cc.h\"", "int main(void) {"]
    for name in STRUCTS:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f in header_struct_fields(name):
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), src, "-o", exe], check=True)
        got = dict(l.split() for l in subprocess.run([exe], stdout=subprocess.PIPE, text=True, check=True)
                   .stdout.splitlines())
    for name in STRUCTS:
        mirror = getattr(_cc, name)
        assert int(got[name]) == ctypes.sizeof(mirror), name
        for f in header_struct_fields(name):
            assert int(got["%s.%s" % (name, f)]) == getattr(mirror, f).offset, (name, f)
