"""The binding's ctypes structures match the C header's: size and every field's offset,
read from a small C program compiled against include/godiet.h with the host compiler."""
import os
import shutil
import subprocess

import pytest

from paper_2211_08157_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [(api.Seqs, "godiet_seqs"), (api.Params, "godiet_sketch_params"),
         (api.Index, "godiet_index"), (api.SeedOpts, "godiet_seed_opts"),
         (api.VoteOpts, "godiet_vote_opts")]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if not shutil.which("gcc") or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("gcc or the HIP headers are missing")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "godiet.h"',
             "int main(void) {"]
    for cls, cname in PAIRS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.parametrize("cls,cname", PAIRS, ids=[c for _, c in PAIRS])
def test_struct_layout_matches_header(c_layout, cls, cname):
    import ctypes
    assert c_layout[(cname, "size")] == ctypes.sizeof(cls)
    for f, _ in cls._fields_:
        assert c_layout[(cname, f)] == getattr(cls, f).offset, f


def test_tuning_keys_are_seed_opts_fields():
    names = [f for f, _ in api.SeedOpts._fields_]
    assert all(k in names for k in api.TUNING_KEYS)
    with pytest.raises(ValueError):
        api.seed_opts(tuning={"no_such_knob": 1})
    o = api.seed_opts(tuning={"long_blocks": 2048, "lookup_blocks": 8192})
    assert (o.long_blocks, o.lookup_blocks, o.long_records, o.shift_mode) == (2048, 8192, 0, -1)
