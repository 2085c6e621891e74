"""Calls from several host threads at once, each on its own stream: the
library keeps no per-call host state beyond per-device caches, so every
result must equal the one-thread result bit for bit."""

import threading

import numpy as np
import pytest
import torch

import latgen
from _gpu import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def _bits(x):
    return torch.view_as_real(x) if x.is_complex() else x


def test_host_threads_on_separate_streams(ops):
    say("concurrency: 4 host threads x 4 streams")
    sites = 20011
    a = to_dev(latgen.random_lattice(sites, seed=81))
    b = to_dev(latgen.random_b(seed=82))
    dc = to_dev(latgen.complex_normal_lattice(sites, seed=83))
    b32 = b.to(torch.complex64)
    packed = {code: ops.pack(a, code) for code in (ops.SU3_F32, ops.SU3_BF16, ops.SU3_R12_F32)}
    a32 = packed[ops.SU3_F32]
    pitch = ops.soa_pitch(sites, ops.SU3_F64)
    torch.cuda.synchronize()

    def work():
        outs = [ops.mult_nn(a, b), ops.mult_na(a, b), ops.mult_an(a, b)]
        outs += [ops.mult_nn(x, b32) for x in packed.values()]
        # SoA: both precisions on the dense layout, FP64 on the padded one,
        # through the transforms each way
        outs += [ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(a), b)),
                 ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(a32), b32)),
                 ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(a, pitch), b, sites=sites), sites)]
        da, db = ops.mult_nn_bwd(a, b, dc)
        return outs + [da, db]

    ref = [x.clone() for x in work()]
    torch.cuda.synchronize()

    results, errors = {}, []

    def run(tid):
        try:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.default_stream())
            with torch.cuda.stream(s):
                last = None
                for _ in range(15):
                    last = work()
            s.synchronize()
            results[tid] = last
        except Exception as e:   # reported below; a thread cannot fail the test itself
            errors.append(repr(e))

    threads = [threading.Thread(target=run, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    torch.cuda.synchronize()
    for tid in range(4):
        for got, want in zip(results[tid], ref):
            assert torch.equal(_bits(got), _bits(want)), "thread %d differs" % tid
