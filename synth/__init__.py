"""Seeded synthetic inputs for the carving scan (master files and disk images).

This package is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It only produces bytes and ground-truth bookkeeping; it computes no
signature, no index and no match (none of the method's arithmetic lives here).
"""
from .workloads import (  # noqa: F401
    CONFIGS,
    FRAGMENT_CONFIGS,
    CarveConfig,
    FragmentConfig,
    DiskImage,
    MasterSet,
    TUNING_IMAGE_ID,
    batch_image_specs,
    batch_images,
    disk_image,
    disk_sectors,
    fragment_files,
    fragment_image,
    fragment_placements,
    master_set,
    master_sectors,
    scaled,
    served_job_slices,
    served_job_specs,
    tuning_sample,
    words,
)
