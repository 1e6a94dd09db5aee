"""mifft: batched 1D FFTs of power-of-two length on MI355X (gfx950): complex-to-complex
(FP32, FP16/BF16) and real-input (R2C / C2R).

The compute path is the C ABI of libmifft.so (include/mifft.h); this package
only marshals arguments.  Importing the package does not load the library:
the first plan does, and it raises if the library has not been built.
"""


def __getattr__(name):
    if name in ("Plan", "RaggedPlan", "fft", "ifft", "FFTFn", "fft_differentiable", "query", "get_plan",
                "weighted_power_loss", "WeightedPowerLossFn", "rfft", "irfft", "RFFTFn", "IRFFTFn",
                "rfft_differentiable", "irfft_differentiable", "PlanND", "fftn", "ifftn", "fft2", "ifft2",
                "FFTNFn", "fftn_differentiable"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
