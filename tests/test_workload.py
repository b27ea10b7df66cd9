"""FLOP accounting of the workloads: the folded count used for the subtree
kernel's roofline drops exactly the per-node multiplies of the first layer's
3E static inputs (R, MCS, SINR: the per-UE part of the actor input of
Sec. VI-B) and adds them back once."""
import pytest

from paper_2506_00167_amd import workload as wl


@pytest.mark.parametrize("cfg", [wl.TINY, wl.TREE_E8K3, wl.STRESS_E16K4, wl.TREE_E8K3.with_head("gaussian")])
def test_folded_flops(cfg):
    E, h1 = cfg.num_ue, cfg.dims[1]
    assert cfg.dims[0] == 4 * E + 2
    assert cfg.flops_per_codebook_folded == cfg.flops_per_codebook - 2 * 3 * E * h1 * (cfg.num_evals - 1)


def test_tree_e8k3_counts():
    c = wl.TREE_E8K3
    assert (c.num_nodes, c.num_evals) == (21845, 16383)
    assert c.flops_per_codebook == 2 * (34 * 256 + 256 * 256 + 256 * 8) * 16383
    assert c.flops_per_codebook_folded == 2 * (10 * 256 + 256 * 256 + 256 * 8) * 16383 + 2 * 24 * 256
