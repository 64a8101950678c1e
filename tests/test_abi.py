"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/*.h, and its host-only logic (variant rules, workspace
sizing, error strings) behaves as documented.  No GPU work is launched."""
import ctypes
import glob
import os
import re

import pytest

from paper_2008_03909_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(cc_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(b.SO_PATH):
        pytest.fail("libconnectit_hip.so is not built")
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(b.SO_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_default_variant_is_the_papers_default():
    v = b.default_variant()
    assert (v.sample, v.kout_k, v.kout_mode) == (b.SAMPLE_KOUT, 2, b.KOUT_HYBRID)
    assert (v.finish, v.splice, v.find) == (b.FIN_UF_REM_CAS, b.SPLICE_SPLIT_ONE, b.FIND_NAIVE)
    assert v.bfs_tries == 3 and abs(v.ldd_beta - 0.2) < 1e-7 and v.ldd_permute == 0


def test_eighty_variants_are_accepted():
    vs = b.all_variants()
    assert len(vs) == 80
    assert len({v.name() for v in vs}) == 80
    for v in vs:
        assert b.check_variant(v) == b.CC_OK, v


def test_extended_variants_are_accepted():
    """UF-Early / UF-Hooks (any find) and label propagation, under every
    sampler, follow the 80 main variants; k-out's max-degree edge choice."""
    vs = b.all_variants(extended=True)
    assert len(vs) == 156 and [v.name() for v in vs[:80]] == [v.name() for v in b.all_variants()]
    assert len({v.name() for v in vs}) == 156
    for v in vs:
        assert b.check_variant(v) == b.CC_OK, v
    assert b.check_variant(b.default_variant(kout_mode=b.KOUT_MAXDEG)) == b.CC_OK
    assert b.check_variant(b.default_variant(kout_mode=4)) == b.CC_EINVAL


def test_rem_with_find_compress_is_rejected():
    """The paper's counter-example combination (Rem + splice + FindCompress) and
    FindCompress with Rem in general are refused."""
    v = b.default_variant()
    for sp in (b.SPLICE_SPLIT_ONE, b.SPLICE_HALVE_ONE, b.SPLICE_ATOMIC):
        assert b.check_variant(v.copy(splice=sp, find=b.FIND_COMPRESS)) == b.CC_EINVAL
    assert b"FindCompress" in b.lib().cc_last_error()
    assert b.check_variant(v.copy(finish=b.FIN_UF_ASYNC, find=b.FIND_COMPRESS)) == b.CC_OK


@pytest.mark.parametrize("field,value,code", [
    ("sample", 7, b.CC_EINVAL), ("kout_k", 0, b.CC_EINVAL), ("finish", 9, b.CC_EINVAL),
    ("find", 5, b.CC_EINVAL), ("splice", 3, b.CC_EINVAL),
])
def test_bad_variant_fields(field, value, code):
    v = b.default_variant()
    setattr(v, field, value)
    assert b.check_variant(v) == code


def test_liu_tarjan_rule_sets():
    """The appendix's 16 combinations are accepted; other rule sets (e.g.
    Connect without Alter, which the appendix notes is incorrect) are not."""
    v = b.default_variant(finish=b.FIN_LT)
    assert len(b.LT_NAMES) == 16
    for r in b.LT_NAMES:
        assert b.check_variant(v.copy(lt_rules=r)) == b.CC_OK
    for r in (b.LT_CONNECT, b.LT_CONNECT | b.LT_FULL_SHORTCUT, b.LT_EXTENDED_CONNECT | b.LT_ROOTUP, 3):
        assert b.check_variant(v.copy(lt_rules=r)) == b.CC_EUNSUPPORTED


def test_workspace_sizes_grow_with_the_variant():
    n, m = 1000, 8000
    base = b.workspace_bytes(n, m, b.default_variant())
    # parent-array scratch, candidate lists, frontier queues and bitmaps
    assert base >= 5 * 4 * n + 3 * n // 8
    bfs = b.workspace_bytes(n, m, b.default_variant(sample=b.SAMPLE_BFS))
    ldd = b.workspace_bytes(n, m, b.default_variant(sample=b.SAMPLE_LDD))
    alt = b.workspace_bytes(n, m, b.default_variant(finish=b.FIN_LT, lt_rules=b.LT_PRFA))
    assert bfs == base and ldd == base        # one layout serves every sampler
    assert alt >= base + 8 * m                # Alter keeps an explicit edge list
    assert b.workspace_bytes(2 * n, 2 * m, b.default_variant()) > base


def test_size_errors():
    sz = ctypes.c_size_t()
    v = b.default_variant()
    L = b.lib()
    assert L.cc_workspace_bytes(0, 0, ctypes.byref(v), ctypes.byref(sz)) == b.CC_EINVAL
    assert L.cc_workspace_bytes(1 << 31, 0, ctypes.byref(v), ctypes.byref(sz)) == b.CC_EINVAL
    assert L.cc_workspace_bytes(10, -1, ctypes.byref(v), ctypes.byref(sz)) == b.CC_EINVAL
    assert L.cc_csr_workspace_bytes(10, 1 << 32, ctypes.byref(sz)) == b.CC_EINVAL
    assert L.cc_status_string(b.CC_ELIVELOCK) == b"CC_ELIVELOCK"


def test_pair_list_workspace_sizing():
    v = b.default_variant()
    sz = ctypes.c_size_t()
    L = b.lib()
    assert L.cc_coo_workspace_bytes(1000, 5000, ctypes.byref(v), ctypes.byref(sz)) == b.CC_OK
    small = sz.value
    # at least the CSR (offsets + 2 * pairs adjacency) and the static workspace
    assert small >= 1001 * 4 + 10000 * 4 + b.workspace_bytes(1000, 10000, v)
    assert L.cc_coo_workspace_bytes(1000, 50000, ctypes.byref(v), ctypes.byref(sz)) == b.CC_OK
    assert sz.value > small
    assert L.cc_coo_workspace_bytes(0, 10, ctypes.byref(v), ctypes.byref(sz)) == b.CC_EINVAL
    assert L.cc_coo_workspace_bytes(10, -1, ctypes.byref(v), ctypes.byref(sz)) == b.CC_EINVAL
    bad = v.copy(find=b.FIND_COMPRESS)
    assert L.cc_coo_workspace_bytes(10, 10, ctypes.byref(bad), ctypes.byref(sz)) == b.CC_EINVAL


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout: gcc
    compiles the header and prints every field's offset and each size."""
    structs = {"cc_variant": b.cc_variant, "cc_amsf_options": b.cc_amsf_options, "cc_stats": b.cc_stats,
               "cc_csr_report": b.cc_csr_report}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "connectit_hip.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, field, val = line.split()
            got[(name, field)] = int(val)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
