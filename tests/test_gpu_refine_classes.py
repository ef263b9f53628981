"""GPU parity of every refinement kernel class against the FP64 oracle: the
FP32 IC-GN and Newton-Raphson kernels are built per slot count (4, 8, 12,
20 and 28 slots of 64 samples per lane, and the two-rows form for 29- and
31-column subsets), and the 20- and 28-slot ones form each sample's offset
from its index instead of keeping it.  Subset radii at the edges of the
classes (a partial last slot, a class's smallest and largest subset), a few
POIs each: integer results and statuses exact, sub-pixel displacements
within 1e-3 px, coefficients within 1e-5 (Sec. 2.2)."""
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# radius -> slots per lane: 3 -> 4, 11 -> 12, 13 -> 12, 16 -> 20, 17 -> 20, 18 -> 28
RADII = [3, 11, 13, 16, 17, 18]


@pytest.mark.parametrize("refine", ["icgn", "nr"])
@pytest.mark.parametrize("M", RADII)
def test_refinement_class(M, refine):
    pr = dicgen.affine_pair_1024(size=160, M=M, S=4, step=11, tag=120 + M)
    pois = pr.pois[:: max(1, len(pr.pois) // 12)]
    slots = ((2 * M + 1) ** 2 + 63) // 64
    print(f"case refine class {refine} M={M} samples/64={slots} N={len(pois)}", flush=True)
    ref = O.correlate(pr.ref, pr.defm, pois, M, pr.S, refine=refine)
    flags = dic.FLAG_REFINE_NR if refine == "nr" else 0
    plan = dic.single_pair_plan(160, 160, M, pr.S, len(pois), dic.FP32_BATCHED, flags=flags)
    out = plan.correlate(to_dev(pr.ref), to_dev(pr.defm), to_dev(pois))
    torch.cuda.synchronize()
    s = compare(host(out), ref, M, label=f"refine class {refine} M={M}")
    assert s["n_ok"] >= len(pois) // 2
