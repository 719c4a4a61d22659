"""slpic_mlp_forward_noalloc (activations in the library's fixed device
array) against slpic_mlp_forward (activations in a caller buffer), through
the C ABI: identical kernels on identical BF16 operands, so the outputs must
be equal bit for bit.  Two calls in a row, the second with a smaller batch
(its result must not depend on what the first left in the array), then the
largest batch the array holds, and a batch beyond it rejected on the host.
Both outputs are also checked against the NumPy oracle of the network."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import mlp
from parity_util import print_case

pytestmark = pytest.mark.gpu


def _params_and_inputs(B, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + 0.02 * rng.normal(size=mlp.N_PARAMS)
    p = p.astype(np.float32).astype(np.float64)
    x = rng.normal(size=(B, 4)).astype(np.float32)
    return p, x


def _reference(gpu_lib, p, x):
    net = gpu_lib.Mlp(p, x.shape[0])
    y = net.forward(x).clone()
    torch.cuda.synchronize()
    return net, y


def test_noalloc_forward_equals_forward_on_two_calls(gpu_lib):
    L = gpu_lib.lib()
    p, x_big = _params_and_inputs(256, 11)
    _, x_small = _params_and_inputs(48, 12)
    net, y_big_ref = _reference(gpu_lib, p, x_big)
    _, y_small_ref = _reference(gpu_lib, p, x_small)
    for name, x, ref in (("first call, batch 256", x_big, y_big_ref), ("second call, batch 48", x_small, y_small_ref)):
        print_case(f"mlp forward_noalloc {name}")
        y = net.forward_noalloc(x)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), name
        yo, _ = mlp.forward(p, x.astype(np.float64), bf16=True)
        yn = y.cpu().numpy().astype(np.float64)
        assert np.abs(yn - yo).max() / np.abs(yo).max() < 2e-3, name
    # the largest batch the fixed array holds
    p2, x_max = _params_and_inputs(gpu_lib.MLP_NOALLOC_MAX_BATCH, 13)
    net2, y_max_ref = _reference(gpu_lib, p2, x_max)
    print_case(f"mlp forward_noalloc batch {gpu_lib.MLP_NOALLOC_MAX_BATCH}")
    y = net2.forward_noalloc(x_max)
    torch.cuda.synchronize()
    assert torch.equal(y, y_max_ref)
    # one batch step beyond it: rejected before any launch
    n = gpu_lib.MLP_NOALLOC_MAX_BATCH + 16
    xo = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    yo = torch.zeros((n, gpu_lib.MLP_OUT), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.slpic_mlp_forward_noalloc(ctypes.c_void_p(net2.pbf16.data_ptr()), ctypes.c_void_p(xo.data_ptr()),
                                     ctypes.c_void_p(yo.data_ptr()), n, stream)
    assert rc == -7 and L.slpic_strerror(rc).decode().startswith("input larger")
    # bad arguments as slpic_mlp_forward
    assert L.slpic_mlp_forward_noalloc(ctypes.c_void_p(net2.pbf16.data_ptr()), ctypes.c_void_p(xo.data_ptr()),
                                       ctypes.c_void_p(yo.data_ptr()), 24, stream) == -1
    torch.cuda.synchronize()
    assert float(yo.abs().max()) == 0.0  # nothing was launched
