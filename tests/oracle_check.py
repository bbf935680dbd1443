"""Comparison of GPU results with the CPU oracle, shared by the GPU tests.

Errors are max-norm errors of each field relative to that field's own
largest magnitude in the reference (psi through |psi|).

float64 state: every field within FP64_TOL of the float64 oracle.

float32 state (every point update still in float64): the GPU result is
compared with two oracle runs from the same float64 inputs,
  * the oracle's float32-storage mode, which rounds the values to float32
    where a float32 state is stored (on entry, after every red sweep, after
    the blue sweep), so that it makes the same roundings from the same
    float32 values: the GPU must equal it up to rare single-ulp rounding
    flips, which arise where the two float64 computations (a different but
    equally accurate complex division) straddle a float32 rounding boundary;
  * the float64 oracle: psi and u within FP32_TOL.  v = u_t picks up the
    float32 rounding of u through the tau*kappa2/h^2 Laplacian of the (u, v)
    update at every step, so its error grows with steps * tau * kappa2 / h^2
    and exceeds FP32_TOL on fine grids whatever a kernel does.  For every
    field the GPU's error against the float64 oracle must equal the error
    that the float32-storage oracle itself makes (the prediction) to within
    a factor of two.
"""
from __future__ import annotations

import numpy as np

import oracle

FP64_TOL = 1e-12
FP32_TOL = 1e-5
# float32 storage emulated: single-ulp rounding flips (2^-24 relative) may
# occur and spread over a few points; this leaves room for a few of them
FP32_EMUL_TOL = 1e-6
PREDICT_BAND = 2.0


def grid_of(p):
    return oracle.Grid(p.dim, p.n, p.lo, p.hi, p.kappa1, p.kappa2, p.mu, p.gamma)


_CACHE = {}


def _key(p, steps, storage_bits):
    import hashlib

    h = hashlib.sha1()
    for a in (p.psi, p.u, p.v):
        h.update(np.ascontiguousarray(a).tobytes())
    return (p.dim, p.n, p.lo, p.hi, p.tau, p.kappa1, p.kappa2, p.mu, p.gamma, steps, storage_bits,
            h.hexdigest())


def oracle_run(p, steps, storage_bits=64, cache=False):
    """The oracle after `steps` steps from p's initial data: the float64
    checkerboard step, or its colour-pass form with float32 storage.  With
    cache=True a result computed before for the same data is reused (tests
    that run one problem under several launch modes)."""
    key = _key(p, steps, storage_bits) if cache else None
    if key is not None and key in _CACHE:
        return _CACHE[key].copy()
    s = oracle.State.from_fields(p.psi, p.u, p.v)
    if storage_bits == 64:
        oracle.step(grid_of(p), p.tau, s, steps)
    else:
        oracle.step_passes(grid_of(p), p.tau, s, steps, storage_bits=storage_bits)
    if key is not None:
        _CACHE[key] = s.copy()
    return s


def fields(x):
    """(psi, u, v) of an oracle State or of a (psi, u, v) tuple."""
    if isinstance(x, oracle.State):
        return x.psi, x.U, x.V
    return tuple(x)


def field_errors(got, ref):
    """Max-norm errors of psi, u and v, each relative to its own field's
    largest magnitude in ref."""
    out = {}
    for name, a, b in zip(("psi", "u", "v"), fields(got), fields(ref)):
        a = np.asarray(a)
        b = np.asarray(b)
        out[name] = float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)
    return out


def compare(precision, got, ref64, ref32=None, label=""):
    """Assert the bar of a state of the given precision against the float64
    oracle result ref64 and, for float32, the float32-storage oracle result
    ref32 (States or (psi, u, v) tuples over the same points); returns the
    errors."""
    err = field_errors(got, ref64)
    if precision == 0:
        print(f"  {label} errors vs float64 oracle:", err, flush=True)
        assert max(err.values()) <= FP64_TOL, (label, err)
        return {"vs_fp64_oracle": err}
    emul = field_errors(got, ref32)
    # a rounding flip of u reaches v through tau*kappa2/h^2: measure the v
    # difference against the larger of the v and u scales
    _, u32, v32 = (np.asarray(a) for a in fields(ref32))
    scale_uv = max(float(np.max(np.abs(v32))), float(np.max(np.abs(u32))))
    emul["v_uv_scale"] = float(np.max(np.abs(np.asarray(fields(got)[2]) - v32))) / scale_uv
    model = field_errors(ref32, ref64)
    print(f"  {label} float32 state: vs float32-storage oracle {emul}; vs float64 oracle "
          f"{err}; predicted {model}", flush=True)
    assert max(emul["psi"], emul["u"], emul["v_uv_scale"]) <= FP32_EMUL_TOL, (label, emul)
    assert err["psi"] <= FP32_TOL and err["u"] <= FP32_TOL, (label, err)
    for f in ("psi", "u", "v"):
        lo, hi = model[f] / PREDICT_BAND, model[f] * PREDICT_BAND
        # below 1e-9 the prediction is a handful of roundings: not a band
        assert lo <= err[f] <= hi or max(err[f], model[f]) <= 1e-9, (label, f, err, model)
    return {"vs_fp64_oracle": err, "vs_fp32_storage_oracle": emul, "predicted": model}


def check(p, got, steps, label="", cache=False):
    """compare() for problem p after `steps` steps from its initial data."""
    ref64 = oracle_run(p, steps, cache=cache)
    ref32 = oracle_run(p, steps, storage_bits=32, cache=cache) if p.precision else None
    return compare(p.precision, got, ref64, ref32, label=label or p.name)
