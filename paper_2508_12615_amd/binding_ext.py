"""Signatures of the optional C ABI groups (graph capture, autotuning, serving).

Declared only for the symbols the loaded library exports, so the core binding
works with any build of libwipes.so.
"""
import ctypes as C


def declare(L) -> None:
    P = C.c_void_p
    table = {}
    for name, (res, args) in table.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
    (P,)
