"""annkin: batched chemical source terms on AMD Instinct MI355X (gfx950).

The hot path (Barwey & Raman, "A Neural Network Inspired Formulation of
Chemical Kinetics", Sec. 2) runs as hand-written HIP kernels in
``libannkin.so`` behind the C ABI of ``include/annkin.h``.  ``annkin`` is the
thin Python binding (argument marshalling only); ``synth`` generates seeded
synthetic mechanisms and states.  Submodules are imported on demand so that
``synth`` stays usable without torch or a GPU.
"""

__all__ = ["annkin", "synth", "build"]
