"""The all-to-all between z-slab shares (paper_1607_00850_amd/slab.py) on
the CPU: where every block lands, for the local copies and for
torch.distributed (gloo, two and three processes).  The layouts come from
hot_plan_slab (host only), so this also checks that the buffers the library
describes tile the workspace the way the exchange assumes."""
import os
import socket

import numpy as np
import pytest
import torch

from paper_1607_00850_amd import binding, slab


def _layouts(N, R, dtype="f32"):
    out = []
    for r in range(R):
        h, ws = binding.hot_plan_slab(N, "rk4", R, r, dtype, nu=0.01, dt=1e-3)
        out.append((binding.hot_slab_layout_of(h), ws))
        binding.hot_destroy(h)
    return out


def _tag(r, c, q, n):
    """Distinct bytes for (source share r, component c, block q)."""
    i = np.arange(n, dtype=np.int64)
    return torch.from_numpy(((i * 7 + r * 31 + c * 17 + q * 5) % 251).astype(np.uint8))


def _fill(ws, lay, offset, ncomp, r):
    v = slab._blocks(ws, lay, offset, ncomp)
    for c in range(ncomp):
        for q in range(lay.nranks):
            v[c, q].copy_(_tag(r, c, q, lay.block_bytes))


def _check(ws, lay, offset, ncomp, r):
    """Block q of component c holds what share q sent for share r."""
    v = slab._blocks(ws, lay, offset, ncomp)
    for c in range(ncomp):
        for q in range(lay.nranks):
            assert torch.equal(v[c, q], _tag(q, c, r, lay.block_bytes)), (r, c, q)


@pytest.mark.parametrize("N,R", [(32, 2), (48, 3), (64, 4)])
def test_exchange_local_moves_every_block(N, R):
    lw = _layouts(N, R)
    wss = [torch.zeros(ws, dtype=torch.uint8) for _, ws in lw]
    lays = [l for l, _ in lw]
    for r in range(R):
        _fill(wss[r], lays[r], lays[r].send_offset, 6, r)
    slab.exchange_local(wss, lays, forward=True)
    for r in range(R):
        _check(wss[r], lays[r], lays[r].recv_offset, 6, r)
    # backward: three components from the receive buffers
    for r in range(R):
        _fill(wss[r], lays[r], lays[r].recv_offset, 3, r)
    slab.exchange_local(wss, lays, forward=False)
    for r in range(R):
        _check(wss[r], lays[r], lays[r].send_offset, 3, r)


def _free_port():
    with socket.socket() as s:
        s.bind(("127.0.0.1", 0))
        return s.getsockname()[1]


def _dist_worker(rank, world, port, N, q):
    import torch.distributed as dist
    os.environ["MASTER_ADDR"] = "127.0.0.1"
    os.environ["MASTER_PORT"] = str(port)
    dist.init_process_group("gloo", rank=rank, world_size=world)
    try:
        h, wsb = binding.hot_plan_slab(N, "rk4", world, rank, "f32", nu=0.01, dt=1e-3)
        lay = binding.hot_slab_layout_of(h)
        binding.hot_destroy(h)
        ws = torch.zeros(wsb, dtype=torch.uint8)
        _fill(ws, lay, lay.send_offset, 6, rank)
        slab.exchange_dist(ws, lay, forward=True)
        _check(ws, lay, lay.recv_offset, 6, rank)
        _fill(ws, lay, lay.recv_offset, 3, rank)
        slab.exchange_dist(ws, lay, forward=False)
        _check(ws, lay, lay.send_offset, 3, rank)
        q.put((rank, "ok"))
    except Exception as e:  # reported to the parent
        q.put((rank, repr(e)))
    finally:
        dist.destroy_process_group()


@pytest.mark.parametrize("N,R", [(32, 2), (48, 3)])
def test_exchange_dist_gloo_matches_the_layout(N, R):
    import torch.multiprocessing as mp
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    port = _free_port()
    procs = [ctx.Process(target=_dist_worker, args=(r, R, port, N, q)) for r in range(R)]
    for p in procs:
        p.start()
    res = dict(q.get(timeout=120) for _ in range(R))
    for p in procs:
        p.join(timeout=60)
    assert res == {r: "ok" for r in range(R)}
