"""Device-resident frames: torch tensors for the inputs and outputs of one frame
and their ``knnf_frame`` view.  Torch only provides the memory and the stream.
"""
from __future__ import annotations

import numpy as np

from . import _lib


class DeviceFrame:
    """Inputs and outputs of one frame on the GPU.

    ``pc1`` (H, W) and ``prob`` (H, W, C) are float32; outputs are allocated
    here: ``out_prob`` (H, W, C) f32, ``out_class`` (H, W) i32 and, with
    ``with_nbr``, ``out_nbr`` (H, W, K) i32 and ``out_dist`` (H, W, K) f32.
    """

    def __init__(self, pc1, prob, K: int, R: int, lam: float, with_nbr: bool = True,
                 device: str = "cuda"):
        import torch

        self.pc1 = torch.as_tensor(np.ascontiguousarray(pc1, np.float32)).to(device)
        self.prob = torch.as_tensor(np.ascontiguousarray(prob, np.float32)).to(device)
        H, W = self.pc1.shape
        C = self.prob.shape[2]
        self.H, self.W, self.C, self.K, self.R, self.lam = H, W, C, int(K), int(R), float(lam)
        self.out_prob = torch.empty((H, W, C), dtype=torch.float32, device=device)
        self.out_class = torch.empty((H, W), dtype=torch.int32, device=device)
        if with_nbr:
            self.out_nbr = torch.empty((H, W, self.K), dtype=torch.int32, device=device)
            self.out_dist = torch.empty((H, W, self.K), dtype=torch.float32, device=device)
        else:
            self.out_nbr = None
            self.out_dist = None

    def as_c(self) -> _lib.knnf_frame:
        f = _lib.knnf_frame()
        f.H, f.W, f.C, f.K, f.R = self.H, self.W, self.C, self.K, self.R
        f.lam = self.lam
        f.pc1 = self.pc1.data_ptr()
        f.prob = self.prob.data_ptr()
        f.out_prob = self.out_prob.data_ptr()
        f.out_class = self.out_class.data_ptr()
        f.out_nbr = self.out_nbr.data_ptr() if self.out_nbr is not None else None
        f.out_dist = self.out_dist.data_ptr() if self.out_dist is not None else None
        return f

    def results(self):
        """Host copies: (out_prob, out_class, nbr or None, dist or None)."""
        return (self.out_prob.cpu().numpy(), self.out_class.cpu().numpy(),
                None if self.out_nbr is None else self.out_nbr.cpu().numpy(),
                None if self.out_dist is None else self.out_dist.cpu().numpy())

    def clear_outputs(self, value: int = 0x7f) -> None:
        """Fill the outputs with a byte pattern (to catch unwritten entries)."""
        import torch

        for t in (self.out_prob, self.out_class, self.out_nbr, self.out_dist):
            if t is not None:
                t.view(torch.uint8).fill_(value)


def current_stream() -> int:
    import torch

    return torch.cuda.current_stream().cuda_stream
