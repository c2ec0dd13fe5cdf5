"""Black-box cross-check against the system OpenSSL command-line tool.

OpenSSL is run as an executable only (``openssl enc``); nothing of it is read
or linked.  It is the one independent implementation of interoperable AES on
this machine, so it pins what the algebraic checks cannot: the S-box affine
constant, the key schedule (RotWord, Rcon) and byte order.  Its CTR mode
increments the whole 16-byte IV as a big-endian integer, which equals the
96-bit nonce || 32-bit big-endian counter layout while the low 32 bits do not
wrap.
"""
from __future__ import annotations

import shutil
import subprocess

OPENSSL = shutil.which("openssl")


def available() -> bool:
    if OPENSSL is None:
        return False
    try:
        r = subprocess.run([OPENSSL, "enc", "-aes-128-ecb", "-nopad", "-K", "00" * 16],
                           input=b"\0" * 16, capture_output=True, timeout=30)
    except (OSError, subprocess.SubprocessError):
        return False
    return r.returncode == 0 and len(r.stdout) == 16


def enc(cipher: str, key: bytes, data: bytes, iv: bytes | None = None, decrypt: bool = False,
        nopad: bool = True) -> bytes:
    cmd = [OPENSSL, "enc", f"-{cipher}", "-K", bytes(key).hex()]
    if nopad:
        cmd.append("-nopad")
    if iv is not None:
        cmd += ["-iv", bytes(iv).hex()]
    if decrypt:
        cmd.append("-d")
    r = subprocess.run(cmd, input=bytes(data), capture_output=True, timeout=120)
    if r.returncode != 0:
        raise RuntimeError(f"openssl failed: {r.stderr.decode(errors='replace')}")
    return r.stdout
