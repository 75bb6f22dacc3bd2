// au_internal.h -- declarations shared by the translation units of the
// library (kernel launch of one trace-length class, validation, errors).
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "aeraunfold.h"
#include "au_kernels.h"

// A pattern table resident on one device, node-major [f][z][a][4] complex.
struct au_table {
    int device;
    int dtype;
    au::GridDev g;
    void* d_nodes;
    size_t bytes;
};

namespace au {

// Records the message for au_last_error() on this thread and returns s.
au_status set_error(au_status s, const std::string& msg);
const std::string& error_string();

constexpr int kStationsPerUnit = 16;
// Batched plans use units of 2 x kStationsPerUnit for events with at least
// this many directions.
constexpr int kWideUnitMinDirs = 64;

struct EvParams {
    int S, N, k_lo, nb;
};

au_status check_common(const au_table* tb, int64_t fs, int64_t lo, int64_t hi, int prec, int tin,
                       double fb, double sg);
au_status check_n(const au_table* tb, int s, int n, int64_t fs, int64_t lo, int64_t hi, EvParams* p);
bool dirs_finite(const double* h, int64_t n);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Unfold-kernel variant currently selected for (precision, N).
int current_variant(int prec, int n);

// One trace-length class of a batch: its event descriptors and work lists
// on the device.
struct ClassLaunch {
    int N = 0;
    int variant = 0;
    const EvDesc* d_evs = nullptr;
    const int2* d_sunits = nullptr;  // (event, station)
    int n_sunits = 0;
    const int2* d_cunits = nullptr;  // (event, direction)
    int n_cunits = 0;
    const int4* d_uunits = nullptr;  // (event, direction, station begin, end)
    int n_uunits = 0;
    unsigned int* d_counter = nullptr;  // non-null: persistent unfold grid (8 counters)
    int persistent_blocks = 0;
    const int* d_xcd_off = nullptr;     // non-null: 8 per-XCD unit lists (9 boundaries)
    int xcd_max_list = 0;               // longest of the 8 lists
    int max_nb = 1 << 30;               // largest band of the events, in bins (default: unknown)
    bool fused = false;                 // spectrum + unfold in one kernel (units: event, station range,
                                        // every direction); needs d_counter
};

// Enqueue spectrum, coefficient and unfold launches of one class on `st`.
// Offsets in the descriptors are relative to the given base pointers.  With
// `stage_events` non-null, an event is recorded after each of the three
// launches.
au_status enqueue_class(const au_table* tb, int prec, int tin, int64_t fs, double fb, double sg,
                        const ClassLaunch& c, const void* volt, void* efield, void* X, void* M,
                        const double* dirs, hipStream_t st, uint64_t* d_counts,
                        hipEvent_t* stage_events);

// Byte sizes of the three parts of the single-event workspace, in order:
// in-band spectra, coefficients, directions (each a multiple of 256).
void workspace_layout(const EvParams& p, int prec, int n_dir, size_t* x_bytes, size_t* m_bytes,
                      size_t* dir_bytes);

// Enqueue the single-event path (spectrum, coefficient and unfold launches,
// the event passed by value) on `st`: d_work is laid out as workspace_layout
// says, its direction part already holding the n_dir directions.
au_status enqueue_event(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                        int n_dir, void* d_efield, void* d_work, hipStream_t st, uint64_t* d_counts);

// Persistent grid size for the unfold kernel of (prec, N, variant).
int persistent_blocks(int prec, int n, int variant, int device);

}  // namespace au
