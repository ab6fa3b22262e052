"""The all-to-all of a z-slab decomposition: moving blocks between shares.

A share's workspace holds a send buffer and a receive buffer, each
[6 components][nranks blocks][nx][N][pitch] elements (hot_slab_layout_of gives
their byte offsets).  After HOT_SLAB_INVERSE the forward exchange moves six
components from the send buffers to the receive buffers; after
HOT_SLAB_CROSS the backward exchange moves three components the other way.
Either way block q of share r's source component lands in block r of share
q's destination component (Sec. 3, "Three dimensional Fourier transforms
with MPI": the Alltoall between the two slab alignments).

The kernels never move these blocks: the collective is the caller's.
exchange_local serves shares that live in one process (device copies);
exchange_dist serves one share per process over torch.distributed, one
all_to_all_single per component (RCCL over xGMI with the "nccl" backend;
"gloo" takes host tensors, so device buffers are staged through host
memory).
"""

FORWARD_COMPONENTS = 6
BACKWARD_COMPONENTS = 3


def _ends(forward):
    if forward:
        return "send_offset", "recv_offset", FORWARD_COMPONENTS
    return "recv_offset", "send_offset", BACKWARD_COMPONENTS


def _blocks(ws, lay, offset, ncomp):
    """Byte view [ncomp][nranks][block_bytes] of a buffer in workspace ws."""
    n = ncomp * lay.comp_bytes
    return ws[offset:offset + n].view(ncomp, lay.nranks, lay.block_bytes)


def exchange_local(workspaces, layouts, forward):
    """All shares in this process: workspaces[r] (uint8 tensors) with
    layouts[r] for share r.  Copies on the tensors' current streams."""
    src_name, dst_name, ncomp = _ends(forward)
    R = len(workspaces)
    for r in range(R):
        lr = layouts[r]
        if lr.rank != r or lr.nranks != R:
            raise ValueError("layouts must be the shares 0..nranks-1 in order")
        src = _blocks(workspaces[r], lr, getattr(lr, src_name), ncomp)
        for q in range(R):
            lq = layouts[q]
            dst = _blocks(workspaces[q], lq, getattr(lq, dst_name), ncomp)
            dst[:, r].copy_(src[:, q])


def exchange_dist(ws, lay, forward, group=None):
    """One share per process (rank lay.rank of a group of lay.nranks):
    torch.distributed.all_to_all_single per component."""
    import torch
    import torch.distributed as dist

    src_name, dst_name, ncomp = _ends(forward)
    if dist.get_world_size(group) != lay.nranks or dist.get_rank(group) != lay.rank:
        raise ValueError("the process group must hold the shares in rank order")
    staged = ws.is_cuda and dist.get_backend(group) == "gloo"
    so, do, cb = getattr(lay, src_name), getattr(lay, dst_name), lay.comp_bytes
    for c in range(ncomp):
        send = ws[so + c * cb:so + (c + 1) * cb]
        recv = ws[do + c * cb:do + (c + 1) * cb]
        if staged:
            torch.cuda.synchronize()
            hs, hr = send.cpu(), torch.empty(cb, dtype=torch.uint8)
            dist.all_to_all_single(hr, hs, group=group)
            recv.copy_(hr)
            torch.cuda.synchronize()
        else:
            dist.all_to_all_single(recv, send, group=group)
