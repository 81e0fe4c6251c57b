"""Teardown order of the Python binding, against a stub library (no GPU):
every handle is destroyed exactly once, plans and servers before their
context when the binding closes them, also when a context and its plan die
together in a reference cycle and at interpreter exit."""
import ctypes
import gc

import pytest

import paper_1804_03807_amd as hp
import workloads as W


class StubLib:
    def __init__(self):
        self.calls = []
        self.next = 100

    def _new(self, ref):
        self.next += 1
        ref._obj.value = self.next
        return 0

    def hp_context_create(self, device, ref):
        self.calls.append(("ctx_create", device))
        return self._new(ref)

    def hp_plan_create(self, ctx, sys, gamma, tol, tune, ref):
        return self._new(ref)

    def hp_server_create(self, ctx, budget, ref):
        return self._new(ref)

    def hp_context_destroy(self, h):
        self.calls.append(("ctx", h.value))

    def hp_plan_destroy(self, h):
        self.calls.append(("plan", h.value))

    def hp_server_destroy(self, h):
        self.calls.append(("server", h.value))

    def hp_path_count(self, sref):
        return 32

    def hp_default_tolerances(self, ref):
        pass


@pytest.fixture
def stub(monkeypatch):
    L = StubLib()
    monkeypatch.setattr(hp, "load", lambda: L)
    return L


def _kinds(L):
    return [c[0] for c in L.calls if c[0] != "ctx_create"]


def test_close_destroys_children_first(stub):
    s = W.dense_small().systems[0]
    ctx = hp.Context(0)
    p = hp.Plan(ctx, s, 1.0)
    srv = hp.Server(ctx, 1 << 30)
    ctx.close()
    kinds = _kinds(stub)
    assert sorted(kinds[:2]) == ["plan", "server"] and kinds[2:] == ["ctx"]
    p.close()
    srv.close()
    ctx.close()
    assert len(_kinds(stub)) == 3  # each handle destroyed once


def test_cycle_collected_together(stub):
    s = W.dense_small().systems[0]
    ctx = hp.Context(0)
    p = hp.Plan(ctx, s, 1.0)
    ctx.cycle = p  # a reference cycle: ctx -> p -> ctx
    del ctx, p
    gc.collect()
    kinds = _kinds(stub)
    assert sorted(kinds) == ["ctx", "plan"]


def test_atexit_hook_closes_children_before_contexts(stub):
    s = W.dense_small().systems[0]
    ctx = hp.Context(0)
    hp.Plan(ctx, s, 1.0)  # only the context holds it (weakly): kept alive here
    keep = hp.Plan(ctx, s, 1.0)
    hp._close_all()
    kinds = _kinds(stub)
    assert kinds[-1] == "ctx" and kinds.count("plan") >= 1 and kinds.count("ctx") == 1
    assert keep.handle is None and ctx.handle is None
