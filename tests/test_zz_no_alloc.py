"""lbm_measure_contact_angle_noalloc (partials in the library's own device array, nothing allocated) against
lbm_measure_contact_angle (partials in the context's workspace) on the same density fields, through the C-ABI: two
calls in a row, the second on a smaller lattice, each bit for bit equal."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1501_05430_amd import workloads as W
from gpu_helpers import gpu_sim

pytestmark = pytest.mark.gpu


def _case(nx, ny, deg, R):
    th = math.radians(deg)
    return W.Case(f"na_{nx}x{ny}", nx, ny, 0.75, np.full(nx, th), np.full(nx, math.pi / 2), [nx / 2],
                  [W.wall_cap_centre(R, th)], [R], 0)


def _noalloc(lib, rho, nx, ny, wall, box, stream):
    b = (C.c_int32 * 4)(*box)
    out = (C.c_double * 5)()
    rc = lib.lbm_measure_contact_angle_noalloc(C.c_void_p(rho.data_ptr()), nx, ny, wall, b,
                                               C.c_void_p(stream.cuda_stream), out)
    return rc, list(out)


def test_noalloc_measurement_equals_the_context_measurement():
    import torch
    import paper_1501_05430_amd as P
    from paper_1501_05430_amd import _lib
    lib = _lib.load()
    for (nx, ny, deg, R, steps, box) in [(256, 128, 60.0, 40.0, 300, (60, 200, 1, 80)),
                                         (128, 64, 120.0, 20.0, 200, (20, 110, 1, 50))]:
        sim = gpu_sim(_case(nx, ny, deg, R), check_every=0)
        sim.step(steps)
        want = sim.measure_contact_angle(box, wall=0)
        rho = sim.rho(device=True)  # the same density field the context measurement reads
        stream = torch.cuda.current_stream()
        rc, got = _noalloc(lib, rho, nx, ny, 0, box, stream)
        assert rc == 0, lib.lbm_last_error().decode()
        assert got[:4] == list(want[:4]) and int(got[4]) == want[4], (got, want)
        # a smaller box on the same field
        small = (box[0] + 10, box[1] - 10, box[2], box[3] - 10)
        want2 = sim.measure_contact_angle(small, wall=0)
        rc, got2 = _noalloc(lib, rho, nx, ny, 0, small, stream)
        assert rc == 0 and got2[:4] == list(want2[:4])
        # the top wall (no droplet there) on both entry points: the same outcome, result or error
        top = (0, nx, ny - 20, ny)
        rc, got3 = _noalloc(lib, rho, nx, ny, 1, top, stream)
        try:
            want3 = sim.measure_contact_angle(top, wall=1)
            assert rc == 0 and got3[:4] == list(want3[:4]), (got3, want3)
        except P.LbmError as e:
            assert rc == e.code
        sim.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_1501_05430_amd import _lib
    lib = _lib.load()
    rho = torch.zeros((10, 10), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    b = (C.c_int32 * 4)(0, 10, 1, 9)
    out = (C.c_double * 5)()
    assert lib.lbm_measure_contact_angle_noalloc(None, 10, 10, 0, b, C.c_void_p(s.cuda_stream), out) == 1
    assert lib.lbm_measure_contact_angle_noalloc(C.c_void_p(rho.data_ptr()), 1, 10, 0, b,
                                                 C.c_void_p(s.cuda_stream), out) == 1
    assert lib.lbm_measure_contact_angle_noalloc(C.c_void_p(rho.data_ptr()), 10, 10, 2, b,
                                                 C.c_void_p(s.cuda_stream), out) == 1
    tiny = (C.c_int32 * 4)(3, 4, 1, 9)
    assert lib.lbm_measure_contact_angle_noalloc(C.c_void_p(rho.data_ptr()), 10, 10, 0, tiny,
                                                 C.c_void_p(s.cuda_stream), out) == 1
