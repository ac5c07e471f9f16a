#!/usr/bin/env python3
"""Writes the stored oracle results of the full-size seeded workloads.

Calls only the seeded input generators (gen/) and the CPU oracle (oracle/).

  stream_u14_<n0>x<n1>x<n2>_seed<s>.txt
      The changes vector a_t (t = 0..16383) of a 14-bit value-noise volume
      too large for one pass of the oracle: the planes are generated chunk by
      chunk on the host, and each chunk, with the plane before it as a
      collar, contributes the cells whose doubled first coordinate q_0 lies
      in [2 z0, 2 z1) (the last chunk also the top layer q_0 = 2 n0).  Every
      cell of the volume is counted exactly once, so the chunk sums add up to
      the whole (Sec. 3, "Streaming" and "Post-Processing"); a chunk's cells
      only touch its own planes and the collar.  The curve is the prefix sum.
  serving_mix_seed4_<n>.txt
      For each request of the serving mix: its dtype, shape, image seed, the
      last curve value and the SHA-256 of its int64 curve (little endian),
      from the oracle on the request's host-generated image.

Usage:
  python tests/golden/make_large_goldens.py stream --shape 1024 8192 8192 --seed 2 [--threads 8]
  python tests/golden/make_large_goldens.py stream --shape 2600 14450 14450 --seed 2 --chunk 4 [--threads 8]
  python tests/golden/make_large_goldens.py serving --count 4096 --seed 4
A stream run keeps its progress in --state (default /tmp/<name>.state.npz)
and resumes from it.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import pathlib
import sys
import time

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parents[1]
sys.path.insert(0, str(ROOT))

import gen  # noqa: E402
import oracle  # noqa: E402

M14 = 16384


def stream_name(shape, seed):
    return f"stream_u14_{shape[0]}x{shape[1]}x{shape[2]}_seed{seed}.txt"


def chunk_vcec(shape, seed, z0, z1, threads):
    """Cells with q_0 in [2 z0, 2 z1) (plus the top layer on the last chunk),
    from planes [max(z0 - 1, 0), z1) generated on the host."""
    n0 = shape[0]
    lo = max(z0 - 1, 0)
    sub = gen.cfg_u14_value_noise(shape, seed=seed, z0=lo, z1=z1)
    off = z0 - lo  # 1 if the collar plane is present
    q_lo = 2 * off
    q_hi = 2 * (off + z1 - z0) + (1 if z1 == n0 else 0)
    return oracle.vcec3_q0_range(sub, M14, q_lo, q_hi, nthreads=threads)


def write_stream(shape, seed, vcec, path, seconds):
    chi = np.cumsum(vcec)
    nz = np.nonzero(vcec)[0]
    digest = hashlib.sha256(chi.astype("<i8").tobytes()).hexdigest()
    with open(path, "w") as f:
        f.write(f"# Changes vector of the 3-D 14-bit value-noise volume {shape[0]} x {shape[1]} x {shape[2]}\n")
        f.write(f"# (uint16 storage; lattice 16, lattice values 0..16383, uniform jitter +-64, seed {seed}),\n")
        f.write("# from the CPU oracle's cell enumeration (Sec. 2, 'Sublevel Set Filtration': a cell's value\n")
        f.write("# is the minimum over its voxels), summed over axis-0 chunks with a one-plane collar\n")
        f.write("# (Sec. 3, 'Streaming', 'Post-Processing').  chi(T_t) = sum of a_s for s <= t.\n")
        f.write(f"# Written by tests/golden/make_large_goldens.py in {seconds:.0f} s.\n")
        f.write(f"shape: {shape[0]} {shape[1]} {shape[2]}\nseed: {seed}\nm: {M14}\n")
        f.write(f"chi_last: {int(chi[-1])}\nchi_sha256: {digest}\nnonzero: {len(nz)}\n")
        for t in nz:
            f.write(f"{int(t)} {int(vcec[t])}\n")


def read_stream(path):
    """(shape, seed, vcec, chi_sha256) of a stored changes vector."""
    shape = seed = digest = None
    vcec = np.zeros(M14, dtype=np.int64)
    for line in pathlib.Path(path).read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        if ":" in line:
            k, v = line.split(":", 1)
            if k == "shape":
                shape = tuple(int(x) for x in v.split())
            elif k == "seed":
                seed = int(v)
            elif k == "chi_sha256":
                digest = v.strip()
            continue
        t, a = line.split()
        vcec[int(t)] = int(a)
    return shape, seed, vcec, digest


def run_stream(shape, seed, chunk, threads, state):
    out = HERE / stream_name(shape, seed)
    state = pathlib.Path(state or f"/tmp/{out.stem}.state.npz")
    n0 = shape[0]
    vcec = np.zeros(M14, dtype=np.int64)
    z = 0
    spent = 0.0
    if state.exists():
        s = np.load(state)
        if tuple(s["shape"]) == tuple(shape) and int(s["seed"]) == seed:
            vcec, z, spent = s["vcec"].copy(), int(s["z"]), float(s["spent"])
            print(f"resuming at plane {z} of {n0}", flush=True)
    while z < n0:
        z1 = min(z + chunk, n0)
        t = time.perf_counter()
        vcec += chunk_vcec(shape, seed, z, z1, threads)
        spent += time.perf_counter() - t
        z = z1
        np.savez(state, shape=np.array(shape), seed=seed, vcec=vcec, z=z, spent=spent)
        print(f"planes [0, {z}) of {n0} done, {spent:.0f} s", flush=True)
    write_stream(shape, seed, vcec, out, spent)
    assert int(vcec.sum()) == 1, "chi at the top threshold must be 1 (the full box is contractible)"
    print(f"wrote {out}", flush=True)


def serving_name(count, seed):
    return f"serving_mix_seed{seed}_{count}.txt"


def run_serving(count, seed, threads):
    reqs = gen.serving_requests(count, seed=seed)
    out = HERE / serving_name(count, seed)
    t0 = time.perf_counter()
    lines = []
    for i, (dtype, shape, iseed) in enumerate(reqs):
        img = gen.serving_image(dtype, shape, iseed)
        m = 256 if dtype == "u8" else M14
        if img.ndim == 3:
            chi = np.cumsum(oracle.vcec3_q0_range(img, m, 0, 2 * img.shape[0] + 1, nthreads=threads))
        else:
            chi = oracle.curve(img, m=m, nthreads=threads)
        digest = hashlib.sha256(chi.astype("<i8").tobytes()).hexdigest()
        lines.append(f"{i} {dtype} {'x'.join(str(s) for s in shape)} {iseed} {int(chi[-1])} {digest}\n")
        if i % 256 == 255:
            print(f"{i + 1} of {count} requests, {time.perf_counter() - t0:.0f} s", flush=True)
    with open(out, "w") as f:
        f.write(f"# Oracle curves of the serving mix (gen.serving_requests({count}, seed={seed})): per request,\n")
        f.write("# index, dtype, shape, image seed, chi at the top threshold and the SHA-256 of the int64 curve\n")
        f.write("# (little endian) from the CPU oracle's cell enumeration (Sec. 2, 'Sublevel Set Filtration').\n")
        f.write(f"# Written by tests/golden/make_large_goldens.py in {time.perf_counter() - t0:.0f} s.\n")
        f.writelines(lines)
    print(f"wrote {out}", flush=True)


def read_serving(path):
    """{index: (dtype, shape, image_seed, chi_last, sha256)}."""
    out = {}
    for line in pathlib.Path(path).read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        i, dtype, shape, iseed, last, digest = line.split()
        out[int(i)] = (dtype, tuple(int(x) for x in shape.split("x")), int(iseed), int(last), digest)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stream", "serving"])
    ap.add_argument("--shape", type=int, nargs=3, default=[1024, 8192, 8192])
    ap.add_argument("--seed", type=int, default=None, help="default: 2 (stream), 4 (serving)")
    ap.add_argument("--chunk", type=int, default=4, help="planes per oracle chunk")
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--state", default=None)
    a = ap.parse_args()
    if a.what == "stream":
        run_stream(tuple(a.shape), 2 if a.seed is None else a.seed, a.chunk, a.threads, a.state)
    else:
        run_serving(a.count, 4 if a.seed is None else a.seed, a.threads)


if __name__ == "__main__":
    main()
