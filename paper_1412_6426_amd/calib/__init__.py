"""HBM counter calibration and rocprofv3 summaries (measurement helpers, not the step)."""
