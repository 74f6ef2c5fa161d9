"""Register budgets of the hot kernels, from the compiler's resource report of
their gfx950 assembly (CPU only: hipcc cross-compiles).

Every schedule is sized for a number of co-resident workgroups per compute
unit; a kernel that grows past the register budget of that count still runs,
only slower or (for the persistent schedules) not at the sizes that need the
count.  Each case states the count the schedule relies on and why."""
import re
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2501_08293_amd import build as B

try:
    B.hipcc()
    _HIPCC = True
except RuntimeError:
    _HIPCC = False

pytestmark = pytest.mark.skipif(not _HIPCC, reason="hipcc not available")

# (source, kernel name prefix of the mangled symbol, minimum wavefronts per SIMD, reason)
CASES = [
    ("admm_persistent.hip", "_ZN3opf22admm_persistent_kernelIfLi4ELb0E", 3,
     "8500-bus FP32 persistent grid: 653 + 1 workgroups of four wavefronts on 256 CUs"),
    ("admm_persistent.hip", "_ZN3opf22admm_persistent_kernelIdLi4ELb0E", 3,
     "8500-bus FP64 persistent grid: 653 + 1 workgroups of four wavefronts on 256 CUs"),
    ("admm_persistent.hip", "_ZN3opf17admm_serve_kernelIfE", 4,
     "FP32 serving launches are sized for four workgroups per CU"),
    ("admm_tiled.hip", "_ZN3opf22admm_tiled_pair_kernelIfLi4E", 4,
     "21000-bus two-tile grid: 810 + 1 workgroups on 256 CUs"),
    ("admm_batch.hip", "_ZN3opf22admm_batch_step_kernelE", 4,
     "batched step kernel: latency-bound, its fourth workgroup per CU is worth 14 % (131 vs 113 us)"),
]


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    d = tmp_path_factory.mktemp("asm")
    srcs = sorted({c[0] for c in CASES})
    with ThreadPoolExecutor(len(srcs)) as ex:
        outs = list(ex.map(lambda s: B.device_assembly(s, str(d / (s + ".s"))), srcs))
    return {s: open(o).read() for s, o in zip(srcs, outs)}


def _resources(text, prefix):
    m = re.search(r"^(" + re.escape(prefix) + r"\S*):", text, re.M)
    assert m, f"kernel {prefix} not found"
    end = text.index(".Lfunc_end", m.end())
    meta = text[end:end + 6000]
    get = lambda k: int(re.search(r"; " + k + r": (\d+)", meta).group(1))
    return {"vgprs": get("TotalNumVgprs"), "occupancy": get("Occupancy"), "scratch": get("ScratchSize")}


@pytest.mark.parametrize("src,prefix,min_waves,why", CASES, ids=[c[1][9:40] for c in CASES])
def test_hot_kernel_keeps_its_occupancy_and_spills_nothing(assembly, src, prefix, min_waves, why):
    r = _resources(assembly[src], prefix)
    assert r["scratch"] == 0, f"{prefix}: {r['scratch']} bytes of register spills per lane"
    assert r["occupancy"] >= min_waves, f"{prefix}: {r['vgprs']} registers allow {r['occupancy']} wavefronts " \
                                        f"per SIMD, the schedule needs {min_waves} ({why})"
