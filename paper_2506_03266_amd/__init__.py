"""MI355X-native synchronous message-passing decoder for the 2D toric code.

Implements the offline decoder of E. Lake, "Fast offline decoding with local
message-passing automata" (arXiv:2506.03266): the message rule A^{(D)} and
feedback F^{(D)} of Def. "message passing automaton, general dimensions"
(Sec. 3.2), run synchronously (Def. "synchronous automaton decoder") on
batches of seeded i.i.d. bit-flip noise samples, as in the numerics of Sec. 7.

Every step of the decode runs in hand-written HIP kernels for gfx950 behind
the C ABI declared in ``include/mpd.h``; :mod:`.binding` marshals torch
tensors to it.  :mod:`.workloads` holds the seeded input recipes.  The
binding is imported lazily so that the input recipes load without a GPU.
"""

__all__ = ["binding", "workloads", "learned", "sweep"]


def __getattr__(name):
    # import_module loads the submodule itself; "from . import name" would ask
    # this hook again for the attribute before importing and recurse.
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
