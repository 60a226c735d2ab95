"""The dense-network sampler's batched-GEMM path replays one captured sweep per
sweep when a call makes two or more sweeps of an even size.  Its results must
equal single-sweep calls (which launch every kernel directly) chained by
resuming from the previous state and step offset, and a second identical call
(which reuses the captured graph) must repeat the first.  Every call goes
through the C interface."""
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    return m


def _say(msg):
    print(msg, flush=True)


def _run(nqs, model, N, C, S, B, seed, dtype, step_offset=0, state=None):
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=seed, dtype=dtype, move="exchange",
                           lanes_per_chain=-1, step_offset=step_offset, init_chains=state is None)
    st = state.clone() if state is not None else torch.empty(C, N, dtype=torch.int8, device=DEV)
    sm = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    lp = torch.empty(S, C, dtype=torch.float32, device=DEV)
    acc = torch.empty(C, dtype=torch.int64, device=DEV)
    nqs.nqs_sample(model, cfg, st, sm, lp, acc)
    return st, sm, lp, acc


@pytest.mark.parametrize("dtype", ["bf16", "e4m3"])
def test_captured_sweeps_equal_direct_launches(nqs, dtype):
    """10x10 Heisenberg, FFNN 100-400-200 on the batched-GEMM path, 512 chains x (2 + 3) exchange sweeps."""
    wl = workloads.cfg3_heis_10x10()
    params = workloads.params_for(wl)
    N, C, B, S = wl.model.n_visible, 512, 2, 3
    model = nqs.Model.from_workload(wl, params)
    _say(f"heis10 {dtype}: one call of {B} + {S} sweeps (graph) against {B + S} single-sweep calls")
    g_st, g_sm, g_lp, g_acc = _run(nqs, model, N, C, S, B, wl.seed, dtype)
    # the same trajectory sweep by sweep: the first call draws the start states, the others resume
    st = None
    sms, lps, acc_sum = [], [], torch.zeros(C, dtype=torch.int64, device=DEV)
    for q in range(B + S):
        st, sm, lp, acc = _run(nqs, model, N, C, 1, 0, wl.seed, dtype, step_offset=q * N, state=st)
        acc_sum += acc
        if q >= B:
            sms.append(sm[0])
            lps.append(lp[0])
    torch.cuda.synchronize()
    assert torch.equal(g_st, st)
    assert torch.equal(g_sm, torch.stack(sms))
    assert torch.equal(g_lp, torch.stack(lps))
    assert torch.equal(g_acc, acc_sum)
    # a second identical call reuses the captured graph and repeats the first
    r_st, r_sm, r_lp, r_acc = _run(nqs, model, N, C, S, B, wl.seed, dtype)
    torch.cuda.synchronize()
    assert torch.equal(r_st, g_st) and torch.equal(r_sm, g_sm) and torch.equal(r_lp, g_lp) and torch.equal(r_acc, g_acc)
    model.close()
