"""The C ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_1104_2732_amd", "libcpselect.so")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                             text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.append(name)
    return names


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("select_kth", "select_kth_ex", "cps_objective", "cps_create", "cps_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks_and_strings():
    import paper_1104_2732_amd as cps
    L = cps.lib()
    assert L.cps_status_string(0) == b"ok"
    assert L.cps_status_string(-1) == b"invalid argument"
    o = cps.default_options()
    assert o.maxit == 64 and o.final_threshold > 0 and 0 < o.partition_fraction <= 1
    # null handle / bad sizes are rejected before any device work
    out = ctypes.c_void_p(0)
    assert L.select_kth(None, None, 10, 1, 0, out, None) == -1
    assert L.select_kth_ex(None, ctypes.c_void_p(16), 0, 1, 0, None, out, None, None) == -1
    assert L.cps_objective(None, ctypes.c_void_p(16), 10, 11, 0, None, 1, out, None) == -1
    assert L.cps_destroy(None) == -1


def test_learned_entry_points_declared():
    names = declared_functions()
    for required in ("cps_mixture_generate", "cps_features", "cps_mlp_forward", "cps_mlp_loss_grad",
                     "cps_mlp_adam", "cps_mlp_init", "cps_learned_bracket", "select_kth_learned",
                     "cps_mlp_train"):
        assert required in names


def test_record_layouts_match_the_binding(tmp_path):
    """sizeof and offsets of the header's records, compiled by the host C compiler, against the
    binding's ctypes mirrors and numpy record types."""
    import subprocess
    import paper_1104_2732_amd as cps
    src = tmp_path / "sizes.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "cpselect.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", '
                   'sizeof(cps_result), sizeof(cps_eval), sizeof(cps_options), '
                   'sizeof(cps_stats), sizeof(cps_batch_options), sizeof(cps_train_options), '
                   'sizeof(cps_train_report), offsetof(cps_options, compact_proposal), '
                   'offsetof(cps_train_options, holdout), sizeof(cps_trim), sizeof(cps_knn), '
                   'offsetof(cps_batch_options, team_capacity)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", HEADER_DIR, "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [cps.RESULT_DTYPE.itemsize, cps.EVAL_DTYPE.itemsize, ctypes.sizeof(cps.Options),
            cps.STATS_DTYPE.itemsize, ctypes.sizeof(cps.BatchOptions),
            ctypes.sizeof(cps.TrainOptions), ctypes.sizeof(cps.TrainReport),
            cps.Options.compact_proposal.offset, cps.TrainOptions.holdout.offset,
            cps.TRIM_DTYPE.itemsize, cps.KNN_DTYPE.itemsize, cps.BatchOptions.team_capacity.offset]
    assert got == want


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_learned_argument_checks():
    import paper_1104_2732_amd as cps
    L = cps.lib()
    p = ctypes.c_void_p(256)
    assert L.cps_mixture_generate(None, 0, 0, 1, 1, p, None, None) == -1
    assert L.cps_features(None, p, p, p, 1, 0, p, p, p, None) == -1
    assert L.cps_mlp_forward(None, p, p, 1, p, None) == -1
    assert L.cps_mlp_loss_grad(None, p, p, p, 1, p, None, None) == -1
    assert L.cps_mlp_adam(None, p, p, p, p, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.cps_mlp_init(None, 0, p, None) == -1
    assert L.cps_learned_bracket(None, p, 10, 1, 0, p, p, None) == -1
    assert L.select_kth_learned(None, p, 10, 1, 0, p, None, p, None, None) == -1
    assert L.cps_mlp_train(None, None, p, None, None) == -1
