"""Host-only checks on the gfx950 assembly of the persistent kernels.

Regression test for a hang: the adjoint kernel once issued a lane-0 atomic at
the end of its item loop, and the compiler threaded that lane guard into the
lane-0 item pop of the next iteration.  The resulting nested loop re-ran the
item-index shuffle with lanes 1..63 only, so those lanes re-processed a stale
item forever.  The kernels must keep exactly one loop around the item pop:
its header issues the counter atomic and no inner loop contains the shuffle
that broadcasts the popped index.  Also checks that the pair kernels use
tiled segment records (vector gathers into LDS, LDS broadcast reads), have a
real branch around the gated beam term and never spill to scratch.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2501_13382_amd", "csrc", "gbs_kernels.hip")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def asm():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    try:
        out = os.path.join(d, "k.s")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-munsafe-fp-atomics", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--offload-device-only", "-S",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(SRC), SRC, "-o", out],
                       check=True, capture_output=True)
        return open(out).read()
    finally:
        shutil.rmtree(d, ignore_errors=True)


def kernels(asm, prefix):
    for m in re.finditer(r"\n(" + prefix + r"[^:\s]*):", asm):
        i = m.start()
        yield m.group(1), asm[i:asm.find(".Lfunc_end", i)], asm[asm.find(".amdhsa_kernel " + m.group(1)):][:4000]


def blocks(body):
    out, cur = {}, None
    for line in body.split("\n"):
        if line.startswith(".LBB"):
            cur = line.split(":")[0]
            out[cur] = [line]
        elif cur:
            out[cur].append(line)
    return out


@pytest.mark.parametrize("prefix", [r"_ZN3gbs7k_pairs", r"_ZN3gbs9k_adjoint"])
def test_single_item_loop_around_pop(asm, prefix):
    found = 0
    for name, body, _ in kernels(asm, prefix):
        found += 1
        bl = blocks(body)
        pop = [b for b, ls in bl.items() if any("global_atomic_add v" in x and "sc0" in x for x in ls)]
        assert len(pop) == 1, (name, pop)
        assert "=>This Loop Header: Depth=1" in bl[pop[0]][0], (name, bl[pop[0]][0])
        depth2 = [b for b, ls in bl.items() if "Loop Header" in ls[0] and "Depth=2" in ls[0]]
        shuffle = [b for b, ls in bl.items() if any("ds_bpermute" in x for x in ls)]
        assert shuffle, name
        first = shuffle[0]
        # the broadcast of the popped index sits directly in the outer loop
        assert "Depth=1" in bl[first][0] and not any(("Header=" + h[1:]) in bl[first][0] for h in depth2), name
    assert found > 0


def test_pair_kernels_tiled_records_real_branch_no_spill(asm):
    for name, body, meta in kernels(asm, r"_ZN3gbs7k_pairs"):
        assert "ds_read_b128" in body and "global_load_dwordx4" in body, name   # tiles: gathered, then LDS
        assert "s_cbranch_vccz" in body or "s_cbranch_execz" in body, name
        m = re.search(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", meta)
        assert m and int(m.group(1)) == 0, name
        for op in ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32"):
            assert op not in body, (name, op)


def _asm_of(source):
    d = tempfile.mkdtemp()
    try:
        out = os.path.join(d, "k.s")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-munsafe-fp-atomics", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--offload-device-only", "-S",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(SRC),
                        os.path.join(os.path.dirname(SRC), source), "-o", out], check=True, capture_output=True)
        return open(out).read()
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("source", ["gbs_kernels.hip", "gbs_trace.hip", "gbs_ir.hip"])
def test_every_kernel_no_scratch_no_packed_fp32(source):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    text = _asm_of(source)
    names = re.findall(r"\.amdhsa_kernel (\S+)", text)
    assert names
    for name in names:
        meta = text[text.find(".amdhsa_kernel " + name):][:4000]
        m = re.search(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", meta)
        assert m and int(m.group(1)) == 0, name
    for op in ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32"):
        assert op not in text, (source, op)


def test_tracer_arithmetic_is_not_contracted():
    """The tracer's table must equal, bit for bit, a reference doing one IEEE
    operation at a time: its only FP64 fused multiply-adds are the ones inside
    correctly rounded divisions (next to v_div_scale / v_div_fmas / v_div_fixup)."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    lines = _asm_of("gbs_trace.hip").split("\n")
    div = [i for i, x in enumerate(lines) if "v_div_scale_f64" in x or "v_div_fmas_f64" in x or "v_div_fixup_f64" in x]
    fmas = [i for i, x in enumerate(lines) if re.search(r"\bv_fmac?_f64", x)]
    assert div and fmas
    for i in fmas:
        assert any(abs(i - j) <= 14 for j in div), lines[i]
