"""The large workload at full size: 1000 VGA frames through a 20 x 20 x 3 m grid of
rooms, 4 mm voxels, 2^22 buckets + 2^19 excess entries, in the plain float form
and the int16 + uint8 form, against the FP64 oracle over the whole stream."""
import numpy as np
import pytest

from synth import make_stream
from tests.gpu_util import compare_raycast, compare_volumes, fuse_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

RAY_FRAMES = (499, 999)


@pytest.fixture(scope="module")
def large_oracle():
    import oracle
    st = make_stream("large")
    print(f"case: large, {st.n_frames} frames generated", flush=True)
    sc = oracle.Scene.from_params(st.params)
    rays, max_vis = {}, 0
    for f in range(st.n_frames):
        sc.integrate(st.depth[f], st.intrinsics, st.T_wc[f])
        max_vis = max(max_vis, sc.stats()["n_visible"])
        if f in RAY_FRAMES:
            rays[f] = sc.raycast(st.width, st.height, st.intrinsics, st.T_wc[f])
        if f % 100 == 0:
            print(f"oracle frame {f}: {sc.stats()}", flush=True)
    return st, sc.export(), sc.stats(), rays, max_vis, sc.export_candidates()


@pytest.mark.parametrize("fmt", ["f32", "s16u8"])
def test_large_full_stream(large_oracle, fmt):
    st, (oc, oF, oW), ostats, orays, max_vis, cands = large_oracle
    print(f"case: large {fmt}", flush=True)
    g, grays, _ = fuse_gpu(st, fmt=fmt, ray_frames=RAY_FRAMES)
    gs = g.stats()
    print(f"gpu stats {gs}; oracle {ostats}; max visible {max_vis}", flush=True)
    assert max_vis <= 2 ** 18
    assert gs["n_allocated"] == ostats["n_allocated"]
    assert gs["n_dropped_total"] == ostats["n_dropped_total"]
    assert gs["n_excess_used"] == ostats["n_excess_used"]
    gc, gF, gW = g.export()
    if fmt == "f32":
        tol = 1e-5
    else:
        def tol(W):
            return (0.5 / 32767 + 4 * 2.0 ** -23) * (np.asarray(W, np.float64) + 1.0) + 1e-6
    compare_volumes((gc, gF, gW), (oc, oF, oW), tol=tol, cands=cands)
    err = np.abs(gF.astype(np.float64) - oF)
    band = (oW > 0) & (np.abs(oF) < 1) & (gW.astype(np.int64) == oW)
    print(f"{fmt}: blocks {len(gc)}, max |dF| {err[band].max():.3e}, rms {np.sqrt(np.mean(err[band] ** 2)):.3e}")
    bar = 0.995 if fmt == "f32" else 0.99
    for f in RAY_FRAMES:
        print(f, compare_raycast(grays[f], orays[f], st.T_wc[f], min_cohit=bar, min_close=bar))
