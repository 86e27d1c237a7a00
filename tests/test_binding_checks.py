"""The Python binding rejects tensors on the wrong device, of the wrong dtype
or shape, before anything reaches the library (a host tensor or a short
buffer would hand a kernel an address it must not read). Runs without a GPU:
the library is replaced by an object that fails if any entry point is called."""
import ctypes
import types

import pytest
import torch

import paper_2504_08339_amd as tn
from paper_2504_08339_amd import _abi, api


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"library entry point {name} reached")


@pytest.fixture
def no_lib(monkeypatch):
    monkeypatch.setattr(api, "_lib", _NoCalls())


def _fake_pop(P=4, n_in=3, n_out=2, N_max=8, C_max=16):
    # a stand-in population on a GPU device (only the fields the checks read)
    return types.SimpleNamespace(P=P, n_in=n_in, n_out=n_out, N_max=N_max, C_max=C_max,
                                 device=torch.device("cuda:0"), c=_abi.TnPopulation(),
                                 t={"conn_w": None, "node_bias": None})


def test_population_needs_gpu_tensors(no_lib):
    ts = {k: torch.zeros((2, 8), dtype=dt) for k, dt in api._NODE.items()}
    ts.update({k: torch.zeros((2, 16), dtype=dt) for k, dt in api._CONN.items()})
    with pytest.raises(ValueError, match="GPU"):
        tn.Population(3, 1, 8, 16, ts)


def test_host_observations_rejected(no_lib):
    pop = _fake_pop()
    for obs in (torch.zeros((5, 3)), torch.zeros((4, 5, 3))):
        with pytest.raises(ValueError, match="must be on"):
            tn.forward(pop, None, obs)
        with pytest.raises(ValueError, match="must be on"):
            tn.backward(pop, None, obs, torch.zeros((4, 5, 2)))


def test_shapes_checked_before_device(monkeypatch, no_lib):
    # pretend host tensors live on the population's device to reach the shape checks
    pop = _fake_pop()
    pop.device = torch.device("cpu")
    with pytest.raises(ValueError, match=r"shape \(5, 3\)"):
        tn.forward(pop, None, torch.zeros((5, 4)))             # wrong n_in
    with pytest.raises(ValueError, match=r"shape \(4, 5, 3\)"):
        tn.forward(pop, None, torch.zeros((3, 5, 3)))          # wrong P
    with pytest.raises(TypeError, match="float32"):
        tn.forward(pop, None, torch.zeros((5, 3), dtype=torch.float64))
    with pytest.raises(TypeError, match="contiguous"):
        tn.forward(pop, None, torch.zeros((3, 5)).t())
    with pytest.raises(ValueError, match="out must have shape"):
        tn.forward(pop, None, torch.zeros((5, 3)), out=torch.zeros((4, 5, 1)))
    obs = torch.zeros((5, 3))
    with pytest.raises(ValueError, match="target must have shape"):
        tn.forward_loss(pop, None, obs, torch.zeros((5, 3)))
    with pytest.raises(ValueError, match="target must have shape"):
        tn.forward_backward_mse(pop, None, obs, torch.zeros((4, 6, 2)))
    with pytest.raises(TypeError, match="float32"):
        tn.forward_backward_mse(pop, None, obs, torch.zeros((5, 2), dtype=torch.float16))
    with pytest.raises(ValueError, match="dY must have shape"):
        tn.backward(pop, None, obs, torch.zeros((4, 5, 3)))


def test_substrate_and_cppn_shapes(no_lib):
    S = 64
    d = torch.device("cpu")
    w1t = torch.zeros((2, S, S), dtype=torch.bfloat16)
    w2t = torch.zeros((2, 8, S), dtype=torch.bfloat16)
    x = torch.zeros((3, S), dtype=torch.bfloat16)
    with pytest.raises(ValueError, match="GPU"):
        tn.substrate_forward(w1t, w2t, x, grid=8)
    pop = _fake_pop(P=2, n_in=5, n_out=1)
    pop.device = d
    with pytest.raises(ValueError, match="dw1t must have shape"):
        tn.cppn_backward(pop, None, torch.zeros((2, S, S + 1)), torch.zeros((2, 8, S)), grid=8)
    with pytest.raises(ValueError, match="dw2t must have shape"):
        tn.cppn_backward(pop, None, torch.zeros((2, S, S)), torch.zeros((2, 7, S)), grid=8)


def test_pack_rejects_host_and_bad_shapes(no_lib):
    with pytest.raises(ValueError, match="GPU"):
        tn.pack_paper_layout(torch.zeros((2, 8, 5)), torch.zeros((2, 16, 4)), 3, 1)


def test_pack_entry_rejects_bad_arguments(monkeypatch):
    lib = _abi.load()
    a = _abi.TnPopulationArrays()
    f = ctypes.cast(ctypes.c_void_p(0x1000), _abi.c_float_p)
    mis = ctypes.cast(ctypes.c_void_p(0x1008), _abi.c_float_p)
    e = ctypes.cast(ctypes.c_void_p(0x2000), _abi.c_int32_p)
    assert lib.tn_pack_paper_layout(f, f, 2, 8, 16, None, e, None) == _abi.TN_EINVAL
    assert lib.tn_pack_paper_layout(f, f, -1, 8, 16, ctypes.byref(a), e, None) == _abi.TN_EINVAL
    assert lib.tn_pack_paper_layout(f, f, 2, 8, 16, ctypes.byref(a), e, None) == _abi.TN_EINVAL
    for name, ty in _abi.TnPopulationArrays._fields_:
        setattr(a, name, ctypes.cast(ctypes.c_void_p(0x3000), ty))
    assert lib.tn_pack_paper_layout(f, mis, 2, 8, 16, ctypes.byref(a), e, None) == _abi.TN_EINVAL
    assert lib.tn_pack_paper_layout(f, f, 2, 8, 16, ctypes.byref(a), None, None) == _abi.TN_EINVAL
    assert lib.tn_pack_paper_layout(f, f, 2, _abi.TN_MAX_NODES + 1, 16, ctypes.byref(a), e,
                                    None) == _abi.TN_EUNSUPPORTED
    assert lib.tn_pack_paper_layout(None, None, 0, 8, 16, ctypes.byref(a), None, None) == _abi.TN_OK
