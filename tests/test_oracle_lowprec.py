"""Why the library's mixed precision stops at float32: an emulation, on the oracle's MINRES, of
P_H^{-1} with the time-axis sine transform (the dense GEMM of Sec. 3.1.1's three-step form)
rounded to float32 or to bfloat16 (operands rounded, float32 accumulation), the spatial
transforms and 1/sigma in float64.  Float32 rounding keeps MINRES within 10% (+1) of the
float64 iteration count; bfloat16 rounding costs more than 10% on every case, so a bfloat16
transform is not built (the GEMMs are only part of a fused launch, so the faster matrix cores
could not repay the extra iterations).  Parity unpinned by design: these are emulations."""
import numpy as np
import pytest

import workloads as W
from oracle.minres import minres
from oracle.sine import dstn, dst_matrix
from oracle.system import System


def _round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _pinv_rounded(s: System, rnd):
    """P_H^{-1} v with the time transforms' GEMMs in the emulated precision."""
    n, N = s.n, s.N
    S = rnd(dst_matrix(n).astype(np.float32))

    def tgemm(X):   # S_n @ X with rounded operands and float32 accumulation
        return (S @ rnd(X.astype(np.float32))).astype(np.float64)

    def apply(v):
        vt = dstn(np.asarray(v, dtype=np.float64).reshape((n, N, N)), (1, 2)).reshape(n, -1)
        zt = tgemm(vt) / s.sigma
        zt = tgemm(zt)
        return dstn(zt.reshape((n, N, N)), (1, 2)).reshape(-1)
    return apply


def test_bf16_rounding_helper():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.14159265, 65504.0], dtype=np.float32)
    r = _round_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie to even
    assert r[2] == np.float32(1.0 + 2 ** -6)     # 1 + 3/256 -> 1 + 4/256 (nearest, 8 mantissa bits)
    assert abs(r[3] + 3.140625) < 1e-12
    assert (r.view(np.uint32) & 0xFFFF).max() == 0


@pytest.mark.parametrize("N,n,theta", [(31, 64, 0.5), (63, 128, 0.5), (31, 128, 1.0)])
def test_bf16_transform_costs_iterations(N, n, theta):
    p = W.crank_nicolson_2d_noisy(N=N, n=n, theta=theta)
    s = System(2, N, n, theta=theta)
    b = s.flip(s.rhs(p.f, p.u0))
    it = {}
    for name, rnd in (("f64", None), ("f32", lambda a: a.astype(np.float32)), ("bf16", _round_bf16)):
        pinv = s.apply_Pinv if rnd is None else _pinv_rounded(s, rnd)
        r = minres(s.apply_YT, pinv, b, rtol=1e-8, maxit=200)
        assert r.status == "converged"
        it[name] = r.iters
    print(f"N={N} n={n} theta={theta}: iterations {it}")
    assert it["f32"] <= int(1.1 * it["f64"]) + 1
    assert it["bf16"] > 1.1 * it["f64"]
