"""Host-side checks of the C ABI library (no GPU needed): it loads, and it
exports every function that include/kv.h and include/kvnn.h declare; the
product package does not import the oracle."""
import ctypes
import os
import re

from paper_2210_08816_amd import kv, kvnn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="kv.h", prefix="kv_"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(kv.ABI_SYMBOLS)
    assert declared_functions("kvnn.h", "kvnn_") == sorted(kvnn.ABI_SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(kv.LIB_PATH):
        from paper_2210_08816_amd import build
        build.build()
    lib = ctypes.CDLL(kv.LIB_PATH)
    for name in declared_functions() + declared_functions("kvnn.h", "kvnn_"):
        assert hasattr(lib, name), name


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2210_08816_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), f
                assert "oracle/" not in src, f


def test_null_context_is_rejected():
    lib = kv.load()
    assert lib.kv_layout(None, None, None) == kv.KV_EINVAL
    assert lib.kv_last_error(None)
    nn = kvnn.load()
    assert nn.kvnn_num_params(None, None) == kvnn.KVNN_EINVAL
    assert nn.kvnn_create(None, None, None) == kvnn.KVNN_EINVAL
    assert nn.kvnn_last_error(None)


def test_bench_dense_transform_model_at_256():
    """The bench's dense-transform roofline model at 256^3: 160 B per cell at
    8 TB/s (0.3355 ms) plus six axis passes at 2 * 256 flop per cell and
    78.6 TFLOP/s (0.6557 ms, above their 96 B per cell at 8 TB/s): 0.991 ms."""
    import bench
    c = 256 ** 3
    t = bench.dense_transform_model_s(c, 256)
    assert abs(t - (160.0 * c / 8e12 + 12.0 * 256 * c / 78.6e12)) < 1e-15
    assert abs(t * 1e3 - 0.991) < 5e-4
