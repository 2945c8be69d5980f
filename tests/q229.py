"""Exact integer total of the stored order-parameter populations of a raw
state buffer (the quantity the 32-bit and 16-bit storage modes conserve
exactly), read from the bytes of the buffer on the host side of the test."""
import torch


def q229_total(raw, precision, nx, ny):
    """Exact integer total of the stored order-parameter populations in a raw
    state buffer (Q2.29 words; binary16 g_1..8 mapped to Q2.29 the way the
    kernels map them)."""
    N = nx * ny
    # plane stride from the buffer size: 18 planes of 4 bytes (FP32) or
    # 17 of 2 bytes + 1 of 4 (FP16 storage)
    Ns = raw.numel() // (72 if precision == "fp32" else 38)
    if precision == "fp32":
        # nine planes of 64-bit words, g_i (Q2.29) in the high 32 bits
        words = raw[:72 * Ns].view(torch.int32).view(9, Ns, 2)[:, :N, 1]
        return int(words.to(torch.int64).sum())
    # FP16 storage: f_0 plane (2 B), g_0 plane (Q2.29 int32), then for
    # i = 1..8 a plane of 32-bit words with g_i in the high half
    g0 = raw[2 * Ns:6 * Ns].view(torch.int32)[:N]
    tot = int(g0.to(torch.int64).sum())
    halves = raw[6 * Ns:38 * Ns].view(torch.float16).view(8, Ns, 2)[:, :N, 1].float()
    for i in range(8):
        scale = 4096.0 if i < 4 else 1024.0
        # the kernels' mapping: the half times 2^29 / scale, truncated
        tot += int(torch.trunc(halves[i] * scale).to(torch.int64).sum())
    return tot
