"""Host logic of the caller-owned workspace (no GPU): it follows what libdk asks for,
which depends on the projector tables as well as on N_s and the expansion degree."""

import torch

from paper_2112_08639_amd import _lib as L
from paper_2112_08639_amd import pipeline


def test_workspace_follows_the_library_size(monkeypatch):
    need = {"bytes": 8000}
    sets = []
    monkeypatch.setattr(L, "dk_workspace_bytes", lambda h, n_s, ng, n_pl: need["bytes"])
    monkeypatch.setattr(L, "dk_set_workspace", lambda h, ws: sets.append(ws.numel() * 8))
    ctx = pipeline.Context.__new__(pipeline.Context)
    ctx.h, ctx.n_grid, ctx.device = object(), 10, torch.device("cpu")
    ctx.ws, ctx.ws_key = None, None

    ctx.ensure_workspace(4, 8)
    assert len(sets) == 1 and sets[0] >= 8000
    # a smaller need (fewer columns) keeps the tensor
    need["bytes"] = 6000
    ctx.ensure_workspace(2, 8)
    assert len(sets) == 1
    # same n_s and degree, but the tables now need more (atoms moved): it grows
    need["bytes"] = 20000
    ctx.ensure_workspace(4, 8)
    assert len(sets) == 2 and sets[1] >= 20000
    assert ctx.ws.numel() * 8 >= 20000
