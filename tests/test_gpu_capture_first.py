"""A plan's very first execution captured in a HIP graph.

The first launch of a pass-B instantiation in a process queries how many of its
workgroups the device holds at once (the kernel takes tiles in turn on that many
resident workgroups).  That query must work inside a stream capture, so this test
runs in a fresh child process, where no pass-B kernel has been launched yet: each
plan's first execution is captured, and every replay must equal an eager call made
afterwards, bit for bit.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child():
    sys.path.insert(0, ROOT)
    import torch
    import paper_1701_04492_amd as P
    from paper_1701_04492_amd import workloads as W
    dev = torch.device("cuda:0")
    for N in (1 << 20, 1 << 22):
        rng = W.rng_for(5)
        x = torch.from_numpy(W.iid_samples(rng, N)).to(dev)
        c = torch.from_numpy(W.complex_normal(rng, N)).to(torch.complex64).to(dev)
        # no autotuning: planning launches no pass-B kernel
        plan = P.nufft2_plan(x, N, 1e-6, torch.complex64, P.NUFFT_FLAG_NO_AUTOTUNE)
        f = torch.empty(N, dtype=torch.complex64, device=dev)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            P.nufft2_exec(plan, c, f)
        outs = []
        for _ in range(3):
            f.zero_()
            _ = (c.abs() + 1).sum().item()   # eager work between replays
            graph.replay()
            torch.cuda.synchronize()
            outs.append(f.clone())
        ref = P.nufft2_exec(plan, c)
        torch.cuda.synchronize()
        ok = [torch.equal(o, ref) for o in outs]
        print("N=%d replays equal to eager: %s" % (N, ok), flush=True)
        if not all(ok):
            sys.exit(1)


def test_first_execution_captured():
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "child"], cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0


if __name__ == "__main__" and sys.argv[1:] == ["child"]:
    _child()
