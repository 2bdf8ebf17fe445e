"""The C ABI library loads and exports every entry point include/kz.h declares (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kz.h")
LIB = os.path.join(ROOT, "paper_2212_00574_amd", "libkz.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kz_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2212_00574_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_entry_points():
    assert declared() == ["kz_batch_autotune", "kz_batch_get_config", "kz_batch_set_config",
                          "kz_batch_workspace_bytes", "kz_clique_workspace_bytes", "kz_colour_jp",
                          "kz_colour_workspace_bytes", "kz_create", "kz_destroy",
                          "kz_dom_workspace_bytes",
                          "kz_dominance", "kz_find_clique", "kz_gen_bitset",
                          "kz_kernelize", "kz_kernelize_async", "kz_kernelize_batch", "kz_kernelize_noalloc", "kz_profile_enable",
                          "kz_profile_read",
                          "kz_server_configure", "kz_server_create", "kz_server_destroy", "kz_server_done", "kz_server_fixed_bytes",
                          "kz_server_poll",
                          "kz_server_progress", "kz_server_request_bytes", "kz_server_submit",
                          "kz_set_edge_path", "kz_strerror", "kz_struction", "kz_struction_workspace_bytes",
                          "kz_workspace_bytes"]


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2212_00574_amd import binding
    assert sorted(binding.EXPORTED) == declared()
    for name in declared():
        assert callable(getattr(binding, name))


def test_status_strings_and_host_argument_checks(lib):
    lib.kz_strerror.restype = C.c_char_p
    assert lib.kz_strerror(0) == b"ok"
    assert b"symmetric" in lib.kz_strerror(-4)
    assert lib.kz_strerror(12345) == b"unknown status"
    # NULL arguments are rejected on the host, before any HIP call
    lib.kz_workspace_bytes.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    assert lib.kz_workspace_bytes(None, None, 3, None) == -1
    lib.kz_create.argtypes = [C.c_void_p, C.c_int]
    assert lib.kz_create(None, 0) == -1


def test_clique_and_colouring_host_checks(lib):
    """Argument checks of the clique search and the colouring that end on
    the host, before the context is touched or any HIP call is made."""
    from paper_2212_00574_amd import binding as b
    lib.kz_clique_workspace_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.kz_find_clique.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.kz_colour_workspace_bytes.argtypes = [C.c_int32, C.c_void_p]
    lib.kz_colour_jp.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]
    g = b.kz_graph(format=b.KZ_BITSET_U64, n=2000, rows=None, row_words=40)
    size = C.c_size_t(0)
    assert lib.kz_clique_workspace_bytes(C.byref(g), 20, C.byref(size)) == b.KZ_OK
    assert size.value >= 2048 * 20 * 40 * 8              # a stack of k * R words per wave
    bigger = C.c_size_t(0)
    assert lib.kz_clique_workspace_bytes(C.byref(g), 21, C.byref(bigger)) == b.KZ_OK and bigger.value > size.value
    assert lib.kz_clique_workspace_bytes(C.byref(g), 65, C.byref(size)) == b.KZ_EINVAL
    dense = b.kz_graph(format=b.KZ_DENSE_U8, n=10)
    assert lib.kz_clique_workspace_bytes(C.byref(dense), 3, C.byref(size)) == b.KZ_EINVAL
    res = b.kz_clique_result()
    fake_ctx = C.create_string_buffer(64)                 # never dereferenced on these paths
    assert lib.kz_find_clique(None, C.byref(g), None, 3, None, None, 0, None, None, C.byref(res)) == b.KZ_EINVAL
    assert res.status == b.KZ_EINVAL
    assert lib.kz_find_clique(fake_ctx, C.byref(dense), None, 3, None, None, 0, None, None, None) == b.KZ_EINVAL
    assert lib.kz_find_clique(fake_ctx, C.byref(g), None, 65, None, None, 0, None, None, None) == b.KZ_ETOOLARGE
    huge = b.kz_graph(format=b.KZ_BITSET_U64, n=1 << 21, rows=None, row_words=1 << 15)
    assert lib.kz_find_clique(fake_ctx, C.byref(huge), None, 3, None, None, 0, None, None,
                              C.byref(res)) == b.KZ_ETOOLARGE and res.status == b.KZ_ETOOLARGE
    assert lib.kz_colour_workspace_bytes(-1, C.byref(size)) == b.KZ_EINVAL
    assert lib.kz_colour_workspace_bytes(1000, C.byref(size)) == b.KZ_OK and size.value >= 1000
    cres = b.kz_colour_result()
    assert lib.kz_colour_jp(None, 10, None, 1, None, None, 0, None, None, C.byref(cres)) == b.KZ_EINVAL
    assert cres.status == b.KZ_EINVAL
    addr = C.c_void_p(1 << 20)                           # 256-byte aligned, never dereferenced here
    assert lib.kz_colour_jp(fake_ctx, 100, addr, 1, addr, addr, 1 << 20, addr, None,
                            None) == b.KZ_EINVAL       # rows narrower than n bits
    assert lib.kz_colour_jp(fake_ctx, 100, addr, 1025, addr, addr, 1 << 20, addr, None,
                            None) == b.KZ_ETOOLARGE    # rows beyond 1024 words
    assert lib.kz_colour_jp(fake_ctx, 100, addr, 2, addr, None, 0, addr, None,
                            None) == b.KZ_EINVAL       # no workspace
    assert lib.kz_colour_jp(fake_ctx, 100, addr, 2, addr, C.c_void_p((1 << 20) + 8), 1 << 20, addr, None,
                            None) == b.KZ_EINVAL       # workspace not 256-byte aligned
    assert lib.kz_colour_jp(None, 0, None, 0, None, None, 0, None, None, None) == b.KZ_EINVAL


def test_product_does_not_reference_the_oracle():
    """The HIP library and its binding never load, link or name the oracle."""
    pkg = os.path.join(ROOT, "paper_2212_00574_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "kz_oracle" not in text and "kzo_" not in text, f


def test_struct_layouts_match_the_header():
    import ctypes as C
    from paper_2212_00574_amd import binding as b
    assert C.sizeof(b.kz_result) == b.RESULT_DTYPE.itemsize == 48
    assert b.BATCH_GRAPH_DTYPE.itemsize == 32
    assert C.sizeof(b.kz_graph) == 56
    assert C.sizeof(b.kz_batch_config) == 20
    assert C.sizeof(b.kz_request) == 48


def test_binding_argument_counts_match_header():
    """Every binding declares as many ctypes arguments as kz.h gives the C
    function parameters (a mismatch would only show at call time)."""
    import re as _re

    from paper_2212_00574_amd import binding
    text = open(os.path.join(ROOT, "include", "kz.h")).read()
    text = _re.sub(r"/\*.*?\*/", " ", text, flags=_re.S)
    for name in declared():
        m = _re.search(r"\b%s\s*\(([^)]*)\)\s*;" % name, text)
        assert m, name
        params = [p for p in m.group(1).split(",") if p.strip() and p.strip() != "void"]
        fn = getattr(binding.LIB, name)
        if fn.argtypes is None:
            continue
        assert len(fn.argtypes) == len(params), (name, len(fn.argtypes), len(params))
