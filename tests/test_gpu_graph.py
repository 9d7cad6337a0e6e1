"""The batched latent step captured in a HIP graph (GPU): the step calls
only enqueue kernels on the caller's stream (no memset, no host read), so a
loop of steps can be captured once and replayed.  Each replay must give the
eager loop's latents and outcomes bit for bit; the replays are separated by
eager work of the program on the same stream and by synchronisations, and
every replay is checked."""
import numpy as np
import pytest

from workloads import Batched2D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("linearized", [True, False])
def test_graph_replay_matches_eager(cuda, linearized):
    import torch
    from paper_2206_02607_amd import crom
    # 96 instances (about 6,900 sample batches): the Gauss-Newton steps take
    # the round-kernel path, as in the 512-instance rollout
    wb = Batched2D(seed=5, n_inst=96)
    dec = crom.Decoder.from_layers(wb.layers, wb.m, precision="bf16", device=cuda)
    st = crom.Stepper(dec, wb.offsets, torch.from_numpy(wb.samples).to(cuda))
    nu = torch.from_numpy(wb.mu).to(cuda)
    opts = crom.GNOptions(max_iter=5, linearized=linearized, tol_step=1e-6)
    K = 4
    q0 = torch.from_numpy(wb.q0).to(cuda)
    # eager reference
    qe = [q0.clone(), torch.empty_like(q0)]
    infos = []
    for i in range(K):
        st.step(qe[i % 2], nu, wb.dt, opts, q_next=qe[(i + 1) % 2])
        infos.append(st.info().copy())
    ref = qe[K % 2].clone()
    torch.cuda.synchronize()
    # capture the K-step loop on static buffers
    q = [q0.clone(), torch.empty_like(q0)]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st.step(q[0], nu, wb.dt, opts, q_next=q[1])  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        for i in range(K):
            st.step(q[i % 2], nu, wb.dt, opts, q_next=q[(i + 1) % 2])
    for rep in range(3):
        q[0].copy_(q0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(q[K % 2], ref), f"replay {rep}"
        assert st.info().tobytes() == infos[-1].tobytes(), f"replay {rep} info"
        # eager work of the program between replays, on the same stream
        st.step(q0, nu, wb.dt, opts, q_next=q[1])
        torch.cuda.synchronize()
