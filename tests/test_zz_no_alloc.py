"""The allocation-free entry point jt_propagate_scratch, through the C ABI:
its posteriors and log Z equal those of jt_bind + jt_propagate in the same
schedule, bit for bit, on two calls in a row (the second on a smaller tree),
and a tree larger than the static scratch is refused without a launch."""
import numpy as np
import pytest

from paper_1202_3777_amd.instances import make_instance

pytestmark = pytest.mark.gpu


def _reference(jt, inst, mode):
    tree = jt.JunctionTree.from_instance(inst)
    tree.propagate(mode)
    outs = [tree.marginals_all(s) for s in range(tree.n_slots)]
    return np.concatenate([o[0] for o in outs]), np.asarray([o[1] for o in outs])


def _scratch(jt, torch, inst, mode):
    plan = jt.JunctionTreePlan.from_instance(inst)
    for s, (v, st) in enumerate(inst.evidence[:plan.n_slots]):
        jt.jt_set_evidence(plan.handle, s, v, st)
    n = int(plan.table_off[-1])
    init = torch.from_numpy(np.ascontiguousarray(inst.potentials)).to("cuda:0")
    post = torch.full((plan.n_slots * n,), -1.0, dtype=torch.float32, device="cuda:0")
    logz = torch.zeros(plan.n_slots, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    jt.jt_propagate_scratch(plan.handle, init.data_ptr(), post.data_ptr(), logz.data_ptr(),
                            jt.MODES[mode], stream.cuda_stream)
    stream.synchronize()
    out = post.cpu().numpy(), logz.cpu().numpy()
    del plan
    return out


def test_scratch_matches_workspace_path():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    cases = [(make_instance("c4", 1, n_slots=4), "fused"),      # batched, shared collect messages
             (make_instance("c1", 2), "fused"),                  # smaller tree, second call
             (make_instance("c1", 2), "plain")]
    for inst, mode in cases:
        need = jt.JunctionTreePlan.from_instance(inst).device_bytes
        print(f"[scratch] {inst.name} slots={inst.n_slots} mode={mode} workspace={need} bytes", flush=True)
        assert need <= 128 << 20
        a, la = _scratch(jt, torch, inst, mode)
        b, lb = _reference(jt, inst, mode)
        assert np.array_equal(a, b), inst.name
        assert np.array_equal(la, lb), inst.name


def test_scratch_refuses_a_tree_too_large():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_3777_amd import jt
    inst = make_instance("c2", 0, n_cliques=40)
    plan = jt.JunctionTreePlan.from_instance(inst)
    assert plan.device_bytes > 128 << 20
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(jt.JTError) as ei:
        jt.jt_propagate_scratch(plan.handle, dummy.data_ptr(), dummy.data_ptr(), dummy.data_ptr(),
                                jt.JT_MODE_FUSED, 0)
    assert ei.value.code == jt.JT_E_NO_MEM
