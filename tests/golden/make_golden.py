"""Write the stored oracle values used by the GPU parity tests.

Calls only ``workloads`` (seeded inputs) and ``oracle`` (CPU reference).
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import direct  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c2_samples():
    """Direct Phi at 64 sampled particles of the 32^3 jittered lattice."""
    x = workloads.jittered_lattice(32768, seed=2)
    idx = workloads.sample_indices(32768, 64, seed=1002)
    t = time.time()
    phi = direct.phi(x, idx)
    out = {
        "workload": "jittered lattice 32^3, spacing 1.0, jitter 0.25, seed 2",
        "n": 32768,
        "sample_seed": 1002,
        "indices": idx.tolist(),
        "phi": [repr(float(v)) for v in phi],
        "oracle_seconds": time.time() - t,
    }
    with open(os.path.join(HERE, "c2_direct_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


def c3_samples(threads: int = 0):
    """Direct Phi at 64 sampled particles of the 262144-point saturated mixture."""
    x = workloads.saturated_gaussian_mixture(262144, seed=3)
    idx = workloads.sample_indices(262144, 64, seed=1003)
    t = time.time()
    phi = direct.phi(x, idx, threads=threads)
    out = {
        "workload": "saturated Gaussian mixture: 32 components, means U[0,100]^3, sigma 2.0, "
                    "min separation 0.3, seed 3",
        "n": 262144,
        "sample_seed": 1003,
        "indices": idx.tolist(),
        "phi": [repr(float(v)) for v in phi],
        "oracle_seconds": time.time() - t,
    }
    with open(os.path.join(HERE, "c3_direct_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


def c3_extra_samples(threads: int = 0, batch: int = 8):
    """Direct Phi at 192 more particles of the 262144-point saturated mixture.

    Together with the 64 of ``c3_samples`` they make 256 sampled particles.
    The extra indices are drawn with seed 2003 from the particles that the
    first 64 do not already hold.  The file is rewritten after every batch of
    ``batch`` particles, so an interrupted run keeps what it has finished and
    a new run continues from there.
    """
    x = workloads.saturated_gaussian_mixture(262144, seed=3)
    first = set(workloads.sample_indices(262144, 64, seed=1003).tolist())
    pool = workloads.sample_indices(262144, 512, seed=2003)
    idx = [int(i) for i in pool if int(i) not in first][:192]
    path = os.path.join(HERE, "c3_direct_samples_extra.json")
    done_i, done_phi, secs = [], [], 0.0
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("planned") == idx:
            done_i, done_phi, secs = old["indices"], old["phi"], old["oracle_seconds"]
    for b in range(len(done_i), len(idx), batch):
        part = idx[b:b + batch]
        t = time.time()
        vals = direct.phi(x, part, threads=threads)
        secs += time.time() - t
        done_i += part
        done_phi += [repr(float(v)) for v in vals]
        out = {
            "workload": "saturated Gaussian mixture: 32 components, means U[0,100]^3, sigma 2.0, "
                        "min separation 0.3, seed 3",
            "n": 262144,
            "sample_rule": "sample_indices(262144, 512, seed=2003) minus the 64 of seed 1003, "
                           "first 192",
            "planned": idx,
            "indices": done_i,
            "phi": done_phi,
            "oracle_seconds": secs,
        }
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)
        print(f"c3 extra: {len(done_i)}/{len(idx)} particles, {secs:.0f} s", flush=True)


def c4_samples(threads: int = 0):
    """Direct Phi at 64 sampled particles of the 16384-point jittered lattice."""
    x = workloads.jittered_lattice(16384, seed=4)
    idx = workloads.sample_indices(16384, 64, seed=1004)
    t = time.time()
    phi = direct.phi(x, idx, threads=threads)
    out = {
        "workload": "jittered lattice, N = 16384 (26^3 sites nearest the centre), spacing 1.0, "
                    "jitter 0.25, seed 4",
        "n": 16384,
        "sample_seed": 1004,
        "indices": idx.tolist(),
        "phi": [repr(float(v)) for v in phi],
        "oracle_seconds": time.time() - t,
    }
    with open(os.path.join(HERE, "c4_direct_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        c2_samples()
    elif which == "c3":
        c3_samples(int(sys.argv[2]) if len(sys.argv) > 2 else 0)
    elif which == "c3x":
        c3_extra_samples(int(sys.argv[2]) if len(sys.argv) > 2 else 0)
    elif which == "c4":
        c4_samples(int(sys.argv[2]) if len(sys.argv) > 2 else 0)
