"""GPU parity of the adjoint kernel against the oracle gradient (itself pinned to finite
differences of the literal measures on the CPU)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2501_03381_amd import api, binding, synth
    binding.lib()
    assert torch.cuda.is_available()
    return torch, api, binding, synth, orc


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_backward_list_latent100(env):
    torch, api, B, synth, orc = env
    X, idx = synth.latent_100(B=600)
    S = orc.gc_covariance(X)
    w = np.random.default_rng(1).standard_normal((4, len(idx)))
    G_ref = orc.grad_list(S, idx, w)
    say("backward LIST N=100 B=600 k 8..20")
    G = api.measures_backward(dev(torch, S), dev(torch, w.astype(np.float32)[:, None, :]), nplets=dev(torch, idx))
    G = G[0].cpu().numpy().astype(np.float64)
    assert np.abs(G - G.T).max() <= 1e-5 * np.abs(G).max()
    assert rel_fro(G, G_ref) < 1e-5


def test_backward_range_and_mask(env):
    torch, api, B, synth, orc = env
    S = orc.gc_covariance(synth.planted_10())
    idx = orc.enumerate_nplets(10, 3, 10)
    w = np.zeros((4, len(idx)))
    w[2] = 1.0                                      # d(sum of Omega) / d Sigma
    G_ref = orc.grad_list(S, idx, w)
    say("backward RANGE N=10 orders 3..10, grad of sum Omega")
    G = api.measures_backward(dev(torch, S), dev(torch, w.astype(np.float32)[:, None, :]), orders=(3, 10))
    assert rel_fro(G[0].cpu().numpy().astype(np.float64), G_ref) < 1e-5
    masks = np.array([sum(1 << int(v) for v in row[row >= 0]) for row in idx], dtype=np.int64)
    say("backward MASK N=10")
    G2 = api.measures_backward(dev(torch, S), dev(torch, w.astype(np.float32)[:, None, :]), masks=dev(torch, masks))
    assert rel_fro(G2[0].cpu().numpy().astype(np.float64), G_ref) < 1e-5


def test_backward_many_datasets_and_not_pd(env):
    torch, api, B, synth, orc = env
    rng = np.random.default_rng(2)
    S = np.stack([synth.random_spd(rng, 12, 50.0) for _ in range(3)])
    S[2, 0, 1] = S[2, 1, 0] = 1.5 * np.sqrt(S[2, 0, 0] * S[2, 1, 1])    # pairs with {0,1} are not PD
    idx = synth.random_nplets(rng, 12, 400, 2, 9)
    w = rng.standard_normal((4, 3, 400))
    say("backward LIST D=3 with not-PD rows")
    G = api.measures_backward(dev(torch, S), dev(torch, w.astype(np.float32)), nplets=dev(torch, idx)).cpu().numpy()
    for d in range(3):
        keep = np.array([orc.is_pd(S[d][np.ix_(r[r >= 0], r[r >= 0])]) for r in idx])
        G_ref = orc.grad_list(S[d], idx[keep], w[:, d, keep])
        assert rel_fro(G[d].astype(np.float64), G_ref) < 1e-5, d


def test_autograd_function(env):
    torch, api, B, synth, orc = env
    S = orc.gc_covariance(synth.planted_10())
    idx = orc.enumerate_nplets(10, 3, 6)
    St = dev(torch, S).requires_grad_(True)
    say("autograd: loss = sum(Omega) + 0.5 sum(S)")
    out = api.nplets_measures_autograd(St, nplets=dev(torch, idx), precision="fp64", out_dtype=torch.float64)
    loss = out[2].sum() + 0.5 * out[3].sum()
    loss.backward()
    w = np.zeros((4, len(idx)))
    w[2], w[3] = 1.0, 0.5
    G_ref = orc.grad_list(S, idx, w)
    assert rel_fro(St.grad.cpu().numpy(), G_ref) < 1e-5
