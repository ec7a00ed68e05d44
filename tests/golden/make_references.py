"""Writes the oracle reference images used by the GPU parity tests.

Only the FP64 oracle (oracle/) is called. The small Cornell box uses O1 (path tracing with
next-event estimation, the plain definition of the path integral). The projector scene uses O3
(plain bidirectional path tracing with every (s, t) strategy): its dim walls are lit through
the lens, and the light paths that reach them there are found by path tracing only when a BSDF
sample happens to hit the small emitter through the lens. The per-pixel sample mean of such an
estimator is skewed, and its variance estimate comes out low exactly where the mean is low,
so O1 at any affordable sample count misreports its own error there. O3 reaches the same paths
by light tracing and vertex connections. Output per scene: per-pixel mean of the per-iteration
pixel values, the variance of that mean, and the number of iterations, as a compressed .npz.

usage: python tests/golden/make_references.py [cfg0|cfg1_128|glass_furnace|glossy_room|all] [spp] [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from synth import scenes  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

REFS = {
    # name: (scene builder, max depth, default spp, oracle method, file tag)
    "cfg0": (lambda: scenes.cornell_glass(64, 64), 8, 262144, 0, "o1"),
    "cfg1_128": (lambda: scenes.projector(128, 128), 12, 8192, 2, "o3"),
    # a lossless glass sphere (IOR 1.5) in an emitting spherical enclosure of albedo 0.5, L_e = 1,
    # depth 120: the closed form L_e / (1 - a) = 2 less the paths the depth limit cuts, which
    # the tessellated sphere makes visible per pixel
    "glass_furnace": (lambda: scenes.furnace(albedo=0.5, le=1.0, glass_sphere=True, width=64, height=64,
                                             sphere_subdiv=2, enclosure="sphere"), 120, 4096, 0, "o1"),
    # the small room with a glossy GGX mirror (roughness 0.1), depth 8, path tracing restricted
    # to the proxy class with specular runs of at most two vertices (what the proxy strategy
    # alone estimates)
    "glossy_room": (lambda: scenes.mirror_room(16, 16, mirror_roughness=0.1), 8, 65536, 0, "o1"),
}
# render options beyond the method and depth
EXTRA = {"glossy_room": dict(u_max=2, class_filter=1)}


def make(name, spp=None, batch=256, threads=None):
    build, depth, default, method, tag = REFS[name]
    spp = spp or default
    S = O.Scene(build())
    s = np.zeros((S.H, S.W, 3))
    s2 = np.zeros((S.H, S.W, 3))
    t0 = time.time()
    for first in range(0, spp, batch):
        n = min(batch, spp - first)
        a, b, _ = S.render(method=method, n_iter=n, first_iter=first, max_depth=depth, seed=12345, threads=threads,
                           **EXTRA.get(name, {}))
        s += a
        s2 += b
        print(f"{name}: {first + n}/{spp} spp, {time.time() - t0:.0f} s", flush=True)
    mean = s / spp
    var_mean = np.maximum(s2 / spp - mean * mean, 0.0) / spp
    out = os.path.join(HERE, f"{name}_{tag}_ref.npz")
    np.savez_compressed(out, mean=mean.astype(np.float64), var_mean=var_mean.astype(np.float64), spp=spp,
                        max_depth=depth, seed=12345, method=method, **EXTRA.get(name, {}))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    spp = int(sys.argv[2]) if len(sys.argv) > 2 and int(sys.argv[2]) > 0 else None
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else None
    for name in (REFS if which == "all" else [which]):
        make(name, spp, threads=threads)
