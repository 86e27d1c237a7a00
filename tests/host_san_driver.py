"""Drives the host-only paths of the C ABI (argument checks, sizes, error
strings) through the AddressSanitizer / UndefinedBehaviorSanitizer build of
the library; run in its own process by test_host_sanitizers.py with the ASan
runtime preloaded. Exits 0 when every call returned the documented status."""
import ctypes
import sys

sys.path.insert(0, sys.argv[2])
from paper_2504_08339_amd import _abi  # noqa: E402

lib = _abi.load(sys.argv[1])
ok = _abi.TN_OK


def fake_pop(**kw):
    p = _abi.TnPopulation()
    p.P, p.n_in, p.n_out, p.N_max, p.C_max = 10, 3, 1, 16, 32
    dummy = ctypes.c_void_p(0x1000)
    for name in ("node_key", "node_bias", "node_resp", "node_act", "node_agg",
                 "conn_in", "conn_out", "conn_w", "conn_en"):
        setattr(p, name, ctypes.cast(dummy, dict(_abi.TnPopulation._fields_)[name]))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def expect(got, want, what):
    if got != want:
        print(f"{what}: got {got}, want {want}", file=sys.stderr)
        sys.exit(1)


for code in range(7):
    lib.tn_status_string(code)
lib.tn_last_error()
expect(lib.tn_validate_population(None), _abi.TN_EINVAL, "null population")
for kw, code in (({}, ok), ({"P": -1}, _abi.TN_EINVAL), ({"N_max": 5000}, _abi.TN_EUNSUPPORTED),
                 ({"n_in": 2000}, _abi.TN_EUNSUPPORTED), ({"node_key": None}, _abi.TN_EINVAL)):
    expect(lib.tn_validate_population(ctypes.byref(fake_pop(**kw))), code, f"validate {kw}")
p = fake_pop()
e = _abi.TnTransformedElems()
expect(lib.tn_transformed_size(ctypes.byref(p), ctypes.byref(e)), ok, "transformed size")
n = ctypes.c_size_t()
for fn in ("tn_distance_workspace_size", "tn_distance_nodes_workspace_size"):
    expect(getattr(lib, fn)(ctypes.byref(p), ctypes.byref(n)), ok, fn)
expect(lib.tn_neat_workspace_size(ctypes.byref(p), 10, ctypes.byref(n)), ok, "neat ws")
expect(lib.tn_neat_workspace_size(ctypes.byref(p), 0, ctypes.byref(n)), _abi.TN_EINVAL, "neat ws 0")
expect(lib.tn_reproduce_workspace_size(1000, ctypes.byref(n)), ok, "reproduce ws")
nu, nz = ctypes.c_int32(), ctypes.c_int32()
expect(lib.tn_reproduce_draws(1024, 4096, ctypes.byref(nu), ctypes.byref(nz)), ok, "draws")
tr = _abi.TnTransformed()
obs = ctypes.cast(ctypes.c_void_p(0x4000), _abi.c_float_p)
expect(lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), obs, 5, 4, None, None), _abi.TN_ESHAPE,
       "forward stride")
expect(lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), obs, 0, 4, None, None), _abi.TN_EINVAL,
       "forward missing transformed")
expect(lib.tn_forward_recurrent(ctypes.byref(p), obs, 0, 4, -1, None, None, None),
       _abi.TN_EINVAL, "recurrent T < 0")
prm = _abi.TnMutationParams(node_add=2.0, n_act_options=1, n_agg_options=1)
arrays = _abi.TnPopulationArrays()
expect(lib.tn_reproduce(ctypes.byref(p), 4, None, None, None, ctypes.byref(prm), 5,
                        ctypes.byref(arrays), None, None, None), _abi.TN_EINVAL, "reproduce")
np_ = _abi.TnNeatParams()
expect(lib.tn_neat_generation(ctypes.byref(p), None, 0, ctypes.byref(np_), None, None, None, None,
                              0, None, None, None, None, None, None), _abi.TN_EINVAL, "neat")
h = ctypes.c_void_p()
expect(lib.tn_plan_create(ctypes.byref(p), ctypes.byref(tr), 4, None, ctypes.byref(h), None),
       _abi.TN_EINVAL, "plan")
lib.tn_plan_destroy(None)
info = _abi.TnBucketInfo()
expect(lib.tn_plan_bucket(None, 0, ctypes.byref(info)), _abi.TN_EINVAL, "plan bucket")
sub = _abi.TnSubstrate(6, 2, 0.2)
expect(lib.tn_substrate_workspace_size(ctypes.byref(sub), 1, 1, 0, ctypes.byref(n)),
       _abi.TN_EUNSUPPORTED, "substrate grid")
for t in ((7, 1, 4, 0), (_abi.TN_ENGINE_REG, 1, 4, 48), (_abi.TN_ENGINE_LDS, 1, 17, 0)):
    tile = _abi.TnTile(*t)
    expect(lib.tn_forward_tiled(ctypes.byref(p), ctypes.byref(tr), obs, 0, 4, None,
                                ctypes.byref(tile), None), _abi.TN_EINVAL, f"tile {t}")
print("host paths clean")
