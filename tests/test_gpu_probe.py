"""The gather-throughput probe (a measurement entry, not part of the method):
it rejects bad arguments, returns a finite positive rate, and a device full of
waves gathers faster than a few waves do."""
import numpy as np
import pytest

from synth import make_config
from helpers import box32

pytestmark = pytest.mark.gpu


def test_gather_probe():
    import gpu_common as gc
    import paper_2303_09916_amd as D
    cfg = make_config(1)
    rec, box = cfg["receptor"], box32(cfg["box"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    torch = g.torch
    ws = gc.dev_bytes(torch, D.dsdp_gather_probe_workspace_bytes(512))
    for blocks, rounds in ((0, 4), (4, 0), (1 << 21, 4), (4, 1 << 17)):
        with pytest.raises(D.DsdpError) as e:
            D.dsdp_gather_probe(g.handle, blocks, rounds, ws)
        assert e.value.status == D.DSDP_ERR_INVALID_ARG
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_gather_probe(g.handle, 513, 4, ws)
    assert e.value.status == D.DSDP_ERR_WORKSPACE_TOO_SMALL
    full = D.dsdp_gather_probe(g.handle, 512, 64, ws)
    few = D.dsdp_gather_probe(g.handle, 4, 64, ws)
    print(f"[gather probe] 2048 waves {full / 1e9:.0f} GB/s, 16 waves {few / 1e9:.0f} GB/s", flush=True)
    assert np.isfinite(full) and np.isfinite(few) and few > 0
    assert full > 4 * few


def test_valu_probe():
    # the FP32 vector-ALU probe: bad arguments rejected; a finite positive rate,
    # no more than the published FP32 vector peak, and a device full of waves
    # issuing far faster than one wave per CU does
    import gpu_common as gc
    import paper_2303_09916_amd as D
    torch = gc.torch_cuda()
    ws = gc.dev_bytes(torch, D.dsdp_gather_probe_workspace_bytes(4096))
    for blocks, iters in ((0, 4), (4, 0), (1 << 21, 4), (4, 1 << 21)):
        with pytest.raises(D.DsdpError) as e:
            D.dsdp_valu_probe(blocks, iters, ws)
        assert e.value.status == D.DSDP_ERR_INVALID_ARG
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_valu_probe(4097, 4, ws)
    assert e.value.status == D.DSDP_ERR_WORKSPACE_TOO_SMALL
    full = max(D.dsdp_valu_probe(4096, 8192, ws) for _ in range(2))
    few = D.dsdp_valu_probe(64, 8192, ws)
    print(f"[valu probe] 16384 waves {full / 1e12:.1f} TFLOP/s, 256 waves {few / 1e12:.1f} TFLOP/s", flush=True)
    assert np.isfinite(full) and np.isfinite(few) and few > 0
    assert full <= 157.3e12 * 1.02 and full > 8 * few
