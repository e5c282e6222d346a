"""Guard words around GPU output buffers: a kernel write past either end of
an output plane changes them."""
import torch

GUARD = 64  # floats (256 bytes) before and after the plane; the plane stays 256-byte aligned
PATTERN = 0x7FC0DEAD  # a quiet-NaN bit pattern no transform of finite inputs produces


def guarded_empty(numel, device="cuda"):
    """(buffer, plane): a float32 buffer of numel + 2 * GUARD words whose
    first and last GUARD words hold PATTERN, and the plane between them."""
    buf = torch.empty(numel + 2 * GUARD, dtype=torch.float32, device=device)
    bits = buf.view(torch.int32)
    bits[:GUARD] = PATTERN
    bits[-GUARD:] = PATTERN
    return buf, buf[GUARD:GUARD + numel]


def assert_guards_intact(buf, name="output"):
    bits = buf.view(torch.int32)
    head_ok = bool((bits[:GUARD] == PATTERN).all())
    tail_ok = bool((bits[-GUARD:] == PATTERN).all())
    assert head_ok and tail_ok, "%s: guard words %s the plane were overwritten" % (
        name, "before" if not head_ok else "after")
